// QR steps of Algorithm 1 (Sec. 3): [Q, R] = qr(G_k^L), G_k <- Q,
// G_{k+1} <- R G_{k+1}^R, and the right-to-left orthogonalisation (LQ of G_k^R
// as the QR of its transpose).  FP64 Householder QR with the LAPACK reflector
// convention (tau = 0 when the column below the diagonal is zero), the
// explicit Q accumulated backwards, and the sign normalisation diag(R) >= 0.
// The operand is read and Q written back through (row, col) strides, so one
// kernel serves both G_k^L and (G_k^R)^T.
//
//  * k_qr_reg: one workgroup, rows in registers (thread t holds rows
//    t + 512 p).  Each reflector takes a single block reduction:
//    ||A[j+1:, j]||^2 and d_c = A[j+1:, j]^T A[j+1:, c], with alpha = A[j][j]
//    and A[j][c] from the thread that holds row j, give beta, tau,
//    v = [1; A[j+1:, j] / (alpha - beta)] and
//    v^T A[:, c] = A[j][c] + d_c / (alpha - beta).  Q is formed in place,
//    backwards, one reduction per reflector.  The wave part of a reduction
//    sums all columns at once by recursive halving (NV - 1 shuffles for NV
//    values), and the column loop is a run-time loop, which keeps the code
//    inside the instruction cache.
//  * k_qr: fallback for operands taller than the registers hold, with the
//    matrix in a global scratch buffer.
#include "tt_internal.h"

namespace {

constexpr int kQrThreads = 1024;

// Reduce NV values per thread across the block; result broadcast in out[0..NV).
template <int NV>
__device__ void block_sum(double (&v)[NV], double* red /* 16*NV */, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, W = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double x = v[q];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[q] = x;
  }
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[w * NV + q] = v[q];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int ww = 0; ww < W; ++ww) s += red[ww * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// A (m x r, col-major, scratch) <- operand; Householder; Q -> operand; R -> Rout (r x r row-major).
__global__ __launch_bounds__(kQrThreads) void k_qr(double* G, int64_t m, int32_t r, int64_t rs, int64_t cs,
                                                  double* __restrict__ A, double* __restrict__ Q,
                                                  double* __restrict__ Rout) {
  __shared__ double red[16 * (TT_MAX_RANK + 1)];
  __shared__ double bc[TT_MAX_RANK + 1];
  __shared__ double tau[TT_MAX_RANK];
  __shared__ double diag[TT_MAX_RANK];
  const int tid = threadIdx.x, T = blockDim.x;
  for (int64_t e = tid; e < m * r; e += T) {
    const int64_t i = e % m, c = e / m;
    A[e] = G[i * rs + c * cs];
  }
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    double* aj = A + (int64_t)j * m;
    // ||A[j+1:, j]||^2
    double v1[1] = {0.0};
    for (int64_t i = j + 1 + tid; i < m; i += T) v1[0] += aj[i] * aj[i];
    block_sum<1>(v1, red, bc);
    const double xnorm2 = bc[0];
    const double alpha = aj[j];
    double beta, t, scale;
    if (xnorm2 == 0.0) {
      t = 0.0;
      beta = alpha;
      scale = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + xnorm2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v = [1; A[j+1:, j] * scale] stored below the diagonal
    if (t != 0.0)
      for (int64_t i = j + 1 + tid; i < m; i += T) aj[i] *= scale;
    __syncthreads();
    if (tid == 0) {
      tau[j] = t;
      diag[j] = beta;
    }
    if (t != 0.0 && j + 1 < r) {
      // w_c = v^T A[j:, c] for c > j, then A[i, c] -= t v_i w_c
      double wv[TT_MAX_RANK];
#pragma unroll
      for (int q = 0; q < TT_MAX_RANK; ++q) wv[q] = 0.0;
      for (int64_t i = j + tid; i < m; i += T) {
        const double vi = i == j ? 1.0 : aj[i];
#pragma unroll
        for (int q = 0; q < TT_MAX_RANK; ++q)
          if (j + 1 + q < r) wv[q] += vi * A[(int64_t)(j + 1 + q) * m + i];
      }
      block_sum<TT_MAX_RANK>(wv, red, bc);
      for (int64_t i = j + tid; i < m; i += T) {
        const double vi = i == j ? 1.0 : aj[i];
#pragma unroll
        for (int q = 0; q < TT_MAX_RANK; ++q)
          if (j + 1 + q < r) A[(int64_t)(j + 1 + q) * m + i] -= t * vi * bc[q];
      }
    }
    __syncthreads();
  }
  // R (before sign normalisation): rows 0..r-1 of the transformed A, diag = beta
  // Q = H_0 ... H_{r-1} [I; 0], accumulated backwards
  for (int64_t e = tid; e < m * r; e += T) {
    const int64_t i = e % m, c = e / m;
    Q[e] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = r - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t == 0.0) continue;   // uniform
    const double* aj = A + (int64_t)j * m;
    double wv[TT_MAX_RANK];
#pragma unroll
    for (int q = 0; q < TT_MAX_RANK; ++q) wv[q] = 0.0;
    for (int64_t i = j + tid; i < m; i += T) {
      const double vi = i == j ? 1.0 : aj[i];
#pragma unroll
      for (int q = 0; q < TT_MAX_RANK; ++q)
        if (q >= j && q < r) wv[q] += vi * Q[(int64_t)q * m + i];
    }
    block_sum<TT_MAX_RANK>(wv, red, bc);
    for (int64_t i = j + tid; i < m; i += T) {
      const double vi = i == j ? 1.0 : aj[i];
#pragma unroll
      for (int q = 0; q < TT_MAX_RANK; ++q)
        if (q >= j && q < r) Q[(int64_t)q * m + i] -= t * vi * bc[q];
    }
    __syncthreads();
  }
  // sign normalisation diag(R) >= 0, write Q to the operand and R out
  for (int64_t e = tid; e < m * r; e += T) {
    const int64_t i = e % m, c = e / m;
    const double sg = diag[c] < 0.0 ? -1.0 : 1.0;
    G[i * rs + c * cs] = sg * Q[e];
  }
  for (int e = tid; e < r * r; e += T) {
    const int i = e / r, c = e - (e / r) * r;
    const double sg = diag[i] < 0.0 ? -1.0 : 1.0;
    double v = 0.0;
    if (c == i) v = diag[i];
    else if (c > i) v = A[(int64_t)c * m + i];
    Rout[e] = sg * v;
  }
}

constexpr int kQrRegThreads = 512;
constexpr int kQrRegWaves = kQrRegThreads / 64;

// Wave sums of NV = 2^L values per lane (L <= 4) by recursive halving: at
// offsets 32, 16, ... a lane keeps one half of its values and adds its
// partner's copy of that half, so L levels take NV - 1 shuffles in all.  Value
// q = lane >> (6 - L) is then summed over the 2^(6-L) lanes that share those
// bits and the wave total returned; every lane of the group holds it.
template <int NV>
__device__ __forceinline__ double wave_sums(double (&v)[NV], int lane) {
#pragma unroll
  for (int half = NV / 2, b = 5; half >= 1; half >>= 1, --b) {
    const bool hi = (lane >> b) & 1;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      double lo = v[i], up = v[i + half];
      // opaque to the optimiser (no instruction): the selects below stay
      // selects of registers instead of becoming a lane-indexed load from a
      // stack copy of v
      asm volatile("" : "+v"(lo), "+v"(up));
      const double keep = hi ? up : lo;
      const double send = hi ? lo : up;
      v[i] = keep + __shfl_xor(send, 1 << b, 64);
    }
  }
  constexpr int L = NV == 1 ? 0 : (NV == 2 ? 1 : (NV == 4 ? 2 : (NV == 8 ? 3 : 4)));
  double x = v[0];
#pragma unroll
  for (int off = 1 << (5 - L); off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Block sums of v[0..NV) over all threads into out[0..NV) (LDS); part is an
// NV x waves LDS buffer.  Two barriers; out is valid after the call.
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* part, double* out) {
  constexpr int L = NV == 4 ? 2 : (NV == 8 ? 3 : 4);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double x = wave_sums<NV>(v, lane);
  if ((lane & ((1 << (6 - L)) - 1)) == 0) part[(lane >> (6 - L)) * kQrRegWaves + wave] = x;
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kQrRegWaves; ++w) s += part[threadIdx.x * kQrRegWaves + w];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Thread t holds rows t + 512 p (p < RPT) of the m x r operand in register
// slots a[p][0..RMAX).  The column loops are run-time loops (the kernel stays
// small enough for the instruction cache), and no slot is ever chosen by a
// run-time index: the factorisation rotates the slots left by one after each
// reflector, so column j is always in slot 0 (columns j + s in slot s, the
// finished Householder vectors behind them), and Q is formed backwards with
// the slots rotated right, so that after the last step slot c holds Q[:, c].
// Each reflector j takes one block reduction of
//   d_s = A[j+1:, j]^T A[j+1:, j+s]   (s = 0 gives ||A[j+1:, j]||^2),
// with row j itself (alpha = A[j][j] and A[j][j+s]) passed through LDS by the
// thread that holds it.  LDS buffers alternate between reductions, so one
// reduction's readers never race the next one's writers.
template <int RMAX, int RPT>
__device__ __forceinline__ void qr_reg_body(gdbl G, int64_t m, int32_t r, int64_t rs, int64_t cs, gdbl __restrict__ Rout) {
  constexpr int NV = RMAX <= 4 ? 4 : (RMAX <= 8 ? 8 : 16);
  static_assert(RMAX <= 16, "register QR holds at most 16 columns");
  __shared__ double part[2][NV * kQrRegWaves];
  __shared__ double fin[2][NV];
  __shared__ double rowj[2][RMAX];
  __shared__ double taus[RMAX], betas[RMAX];
  const int tid = threadIdx.x;
  double a[RPT][RMAX];
#pragma unroll
  for (int p = 0; p < RPT; ++p) {
    const int64_t i = tid + (int64_t)kQrRegThreads * p;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[p][c] = (i < m && c < r) ? G[i * rs + c * cs] : 0.0;
  }
  int buf = 0;
  // ---- factorisation
  for (int j = 0; j < r; ++j) {
    if (tid == j)
#pragma unroll
      for (int s = 0; s < RMAX; ++s) rowj[buf][s] = a[0][s];
    double v[NV], x[RPT];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int64_t i = tid + (int64_t)kQrRegThreads * p;
      x[p] = (i > j && i < m) ? a[p][0] : 0.0;
#pragma unroll
      for (int s = 0; s < RMAX; ++s) v[s] += x[p] * a[p][s];
    }
    block_sums<NV>(v, part[buf], fin[buf]);
    const double alpha = rowj[buf][0], xnorm2 = fin[buf][0];
    double t = 0.0, bt = alpha, scale = 0.0;
    if (xnorm2 != 0.0) {
      const double nrm = sqrt(alpha * alpha + xnorm2);
      bt = alpha >= 0.0 ? -nrm : nrm;
      t = (bt - alpha) / bt;
      scale = 1.0 / (alpha - bt);
    }
    if (tid == 0) {
      taus[j] = t;
      betas[j] = bt;
    }
    // A[:, j+s] -= t v (v^T A[:, j+s]) for 0 < s < r - j, v = [1; A[j+1:, j] scale]
#pragma unroll
    for (int s = 1; s < RMAX; ++s) {
      if (s < r - j) {
        const double wc = rowj[buf][s] + scale * fin[buf][s];
#pragma unroll
        for (int p = 0; p < RPT; ++p) {
          const int64_t i = tid + (int64_t)kQrRegThreads * p;
          a[p][s] -= (i == j ? t : t * x[p] * scale) * wc;   // x = 0 outside rows j+1..m-1
        }
      }
    }
    // column j: beta on the diagonal, the Householder vector below it; then
    // rotate so that column j + 1 comes to slot 0
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int64_t i = tid + (int64_t)kQrRegThreads * p;
      const double c0 = i == j ? bt : (i > j ? x[p] * scale : a[p][0]);
#pragma unroll
      for (int s = 0; s + 1 < RMAX; ++s) a[p][s] = a[p][s + 1];
      a[p][RMAX - 1] = c0;
    }
    buf ^= 1;
  }
  __syncthreads();   // taus / betas
  // ---- R with diag(R) >= 0 (row i lives in thread i, slot 0, for i < r <= 16);
  // slot s now holds column (r + s) mod RMAX
  if (tid < r) {
    const double sg = betas[tid] < 0.0 ? -1.0 : 1.0;
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int c = (r + s) % RMAX;
      if (c < r) Rout[tid * r + c] = c < tid ? 0.0 : sg * (c == tid ? betas[tid] : a[0][s]);
    }
  }
  // ---- explicit Q in place, backwards: Q <- H_j Q.  After the right
  // rotation slot 0 holds the vector of reflector j and slots 1..r-1-j the Q
  // columns j+1..r-1 formed so far.
  for (int j = r - 1; j >= 0; --j) {
    const double t = taus[j];
    double vi[RPT];
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const double last = a[p][RMAX - 1];
#pragma unroll
      for (int s = RMAX - 1; s > 0; --s) a[p][s] = a[p][s - 1];
      a[p][0] = last;
      const int64_t i = tid + (int64_t)kQrRegThreads * p;
      vi[p] = i == j ? 1.0 : ((i > j && i < m) ? a[p][0] : 0.0);
    }
    if (j < r - 1) {
      double v[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] = 0.0;
#pragma unroll
      for (int p = 0; p < RPT; ++p)
#pragma unroll
        for (int s = 1; s < RMAX; ++s)
          if (s < r - j) v[s] += vi[p] * a[p][s];
      block_sums<NV>(v, part[buf], fin[buf]);
#pragma unroll
      for (int s = 1; s < RMAX; ++s)
        if (s < r - j) {
          const double wc = fin[buf][s];
#pragma unroll
          for (int p = 0; p < RPT; ++p) a[p][s] -= t * vi[p] * wc;
        }
      buf ^= 1;
    }
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int64_t i = tid + (int64_t)kQrRegThreads * p;
      a[p][0] = i > j ? -t * vi[p] : (i == j ? 1.0 - t : 0.0);
    }
  }
  // ---- Q with the column signs of the normalisation (slot c = column c)
#pragma unroll
  for (int p = 0; p < RPT; ++p) {
    const int64_t i = tid + (int64_t)kQrRegThreads * p;
    if (i < m)
#pragma unroll
      for (int c = 0; c < RMAX; ++c)
        if (c < r) G[i * rs + c * cs] = (betas[c] < 0.0 ? -1.0 : 1.0) * a[p][c];
  }
}

template <int RMAX, int RPT>
__global__ __launch_bounds__(kQrRegThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_qr_reg(double* G, int64_t m, int32_t r, int64_t rs, int64_t cs,
                                                         double* __restrict__ Rout) {
  qr_reg_body<RMAX, RPT>((gdbl)G, m, r, rs, cs, (gdbl)Rout);
}

// Batched: QR of G_k^L (R_k n_k x R_{k+1}) of problem idx[blockIdx.x].
template <int RMAX, int RPT>
__global__ __launch_bounds__(kQrRegThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) void kb_qr(const BUpd* __restrict__ d, const int32_t* __restrict__ idx) {
  const BUpd u = d[idx[blockIdx.x]];
  const int64_t m = (int64_t)u.rk * u.nk;
  qr_reg_body<RMAX, RPT>((gdbl)u.G, m, u.rk1, 1, m, (gdbl)u.R);
}

// Batched: QR of G_s^R transposed (m x r, row stride r) of problem
// idx[blockIdx.x], R into the problem's R buffer.
template <int RMAX, int RPT>
__global__ __launch_bounds__(kQrRegThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) void kb_qr_right(const BRo* __restrict__ d, const int32_t* __restrict__ idx) {
  const BRo u = d[idx[blockIdx.x]];
  qr_reg_body<RMAX, RPT>((gdbl)u.G, u.m, u.r, u.r, 1, (gdbl)u.R);
}

template <int RMAX>
hipError_t qr_reg(const tt_plan_s* p, double* G, int64_t m, int64_t r, int64_t rs, int64_t cs) {
  double* R = p->at<double>(p->o_qrR);
  const dim3 grid(1), block(kQrRegThreads);
  const int32_t ri = (int32_t)r;
  if (m <= kQrRegThreads) hipLaunchKernelGGL((k_qr_reg<RMAX, 1>), grid, block, 0, p->stream, G, m, ri, rs, cs, R);
  else if (m <= 2 * kQrRegThreads) hipLaunchKernelGGL((k_qr_reg<RMAX, 2>), grid, block, 0, p->stream, G, m, ri, rs, cs, R);
  else if (m <= 4 * kQrRegThreads) hipLaunchKernelGGL((k_qr_reg<RMAX, 4>), grid, block, 0, p->stream, G, m, ri, rs, cs, R);
  else if constexpr (RMAX <= 12) hipLaunchKernelGGL((k_qr_reg<RMAX, 8>), grid, block, 0, p->stream, G, m, ri, rs, cs, R);
  else return hipErrorInvalidValue;   // not reached: launch_qr_core routes these shapes to k_qr
  return hipGetLastError();
}

// G^R (r x cols, column-major, ld r) <- R G^R; thread per column.
__global__ void k_absorb_left(double* G, const double* __restrict__ R, int32_t r, int64_t cols) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= cols) return;
  double x[TT_MAX_RANK];
#pragma unroll
  for (int q = 0; q < TT_MAX_RANK; ++q) x[q] = q < r ? G[p * r + q] : 0.0;
#pragma unroll
  for (int a = 0; a < TT_MAX_RANK; ++a) {
    if (a < r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < TT_MAX_RANK; ++q)
        if (q < r) acc += R[a * r + q] * x[q];
      G[p * r + a] = acc;
    }
  }
}

// Batched: G_{k+1}^R <- R G_{k+1}^R for problem blockIdx.y.
__global__ void kb_absorb_left(const BUpd* __restrict__ d) {
  const BUpd u = d[blockIdx.y];
  if (!u.Gnext) return;
  const gdbl Gn = (gdbl)u.Gnext;
  const cgdbl Rg = (cgdbl)u.R;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= u.ncols_next) return;
  const int r = u.rk1;
  double x[TT_MAX_RANK];
#pragma unroll
  for (int q = 0; q < TT_MAX_RANK; ++q) x[q] = q < r ? Gn[p * r + q] : 0.0;
#pragma unroll
  for (int a = 0; a < TT_MAX_RANK; ++a) {
    if (a < r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < TT_MAX_RANK; ++q)
        if (q < r) acc += Rg[a * r + q] * x[q];
      Gn[p * r + a] = acc;
    }
  }
}

// G^L (rows x r, column-major, ld rows) <- G^L R^T; thread per row.
__global__ void k_absorb_right(double* G, const double* __restrict__ R, int64_t rows, int32_t r) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= rows) return;
  double x[TT_MAX_RANK];
#pragma unroll
  for (int q = 0; q < TT_MAX_RANK; ++q) x[q] = q < r ? G[p + rows * q] : 0.0;
#pragma unroll
  for (int b = 0; b < TT_MAX_RANK; ++b) {
    if (b < r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < TT_MAX_RANK; ++q)
        if (q < r) acc += x[q] * R[b * r + q];
      G[p + rows * b] = acc;
    }
  }
}

// Batched: G_{s-1}^L <- G_{s-1}^L R^T for problem blockIdx.y (thread per row).
__global__ void kb_absorb_right(const BRo* __restrict__ d) {
  const BRo u = d[blockIdx.y];
  if (!u.Gprev) return;
  const gdbl G = (gdbl)u.Gprev;
  const cgdbl Rg = (cgdbl)u.R;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= u.rows) return;
  const int r = u.r;
  const int64_t rows = u.rows;
  double x[TT_MAX_RANK];
#pragma unroll
  for (int q = 0; q < TT_MAX_RANK; ++q) x[q] = q < r ? G[p + rows * q] : 0.0;
#pragma unroll
  for (int b = 0; b < TT_MAX_RANK; ++b) {
    if (b < r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < TT_MAX_RANK; ++q)
        if (q < r) acc += x[q] * Rg[b * r + q];
      G[p + rows * b] = acc;
    }
  }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_qr_core(const tt_plan_s* p, double* G, int64_t m, int64_t rcols, int64_t rs, int64_t cs) {
  if (m <= 4 * kQrRegThreads || (m <= 8 * kQrRegThreads && rcols <= 12)) {
    if (rcols <= 4) return qr_reg<4>(p, G, m, rcols, rs, cs);
    if (rcols <= 8) return qr_reg<8>(p, G, m, rcols, rs, cs);
    if (rcols <= 12) return qr_reg<12>(p, G, m, rcols, rs, cs);
    return qr_reg<16>(p, G, m, rcols, rs, cs);
  }
  hipLaunchKernelGGL(k_qr, dim3(1), dim3(kQrThreads), 0, p->stream, G, m, (int32_t)rcols, rs, cs,
                     p->at<double>(p->o_qrA), p->at<double>(p->o_qrQ), p->at<double>(p->o_qrR));
  return hipGetLastError();
}

hipError_t launch_absorb_left(const tt_plan_s* p, double* Gnext, int64_t r, int64_t cols) {
  hipLaunchKernelGGL(k_absorb_left, dim3(nblk(cols, 256)), dim3(256), 0, p->stream, Gnext, p->at<double>(p->o_qrR),
                     (int32_t)r, cols);
  return hipGetLastError();
}

hipError_t launch_absorb_right(const tt_plan_s* p, double* Gprev, int64_t rows, int64_t r) {
  hipLaunchKernelGGL(k_absorb_right, dim3(nblk(rows, 256)), dim3(256), 0, p->stream, Gprev, p->at<double>(p->o_qrR),
                     rows, (int32_t)r);
  return hipGetLastError();
}

template <int RMAX, int RPT>
hipError_t qr_batched_t(const BUpd* d, const int32_t* idx, int32_t nidx, hipStream_t st) {
  hipLaunchKernelGGL((kb_qr<RMAX, RPT>), dim3((unsigned)nidx), dim3(kQrRegThreads), 0, st, d, idx);
  return hipGetLastError();
}

template <int RMAX>
hipError_t qr_batched_r(const BUpd* d, const int32_t* idx, int32_t nidx, int32_t rpt, hipStream_t st) {
  if (rpt <= 1) return qr_batched_t<RMAX, 1>(d, idx, nidx, st);
  if (rpt <= 2) return qr_batched_t<RMAX, 2>(d, idx, nidx, st);
  return qr_batched_t<RMAX, 4>(d, idx, nidx, st);
}

// Problems of one class (RMAX >= R_{k+1}, RPT * 512 >= R_k n_k, at most 4 rows
// per thread) in one launch.
hipError_t launch_qr_batched(const BUpd* d, const int32_t* idx, int32_t nidx, int32_t rmax, int32_t rpt, hipStream_t st) {
  if (nidx <= 0) return hipSuccess;
  if (rpt > 4) return hipErrorInvalidValue;
  if (rmax <= 4) return qr_batched_r<4>(d, idx, nidx, rpt, st);
  if (rmax <= 8) return qr_batched_r<8>(d, idx, nidx, rpt, st);
  if (rmax <= 12) return qr_batched_r<12>(d, idx, nidx, rpt, st);
  return qr_batched_r<16>(d, idx, nidx, rpt, st);
}

hipError_t launch_absorb_left_batched(const BUpd* d, int32_t nprob, int32_t max_cols, hipStream_t st) {
  if (nprob <= 0 || max_cols <= 0) return hipSuccess;   // last step: no problem has a next core
  hipLaunchKernelGGL(kb_absorb_left, dim3(nblk(max_cols, 256), (unsigned)nprob), dim3(256), 0, st, d);
  return hipGetLastError();
}

template <int RMAX, int RPT>
hipError_t qr_right_t(const BRo* d, const int32_t* idx, int32_t nidx, hipStream_t st) {
  hipLaunchKernelGGL((kb_qr_right<RMAX, RPT>), dim3((unsigned)nidx), dim3(kQrRegThreads), 0, st, d, idx);
  return hipGetLastError();
}

template <int RMAX>
hipError_t qr_right_r(const BRo* d, const int32_t* idx, int32_t nidx, int32_t rpt, hipStream_t st) {
  if (rpt <= 1) return qr_right_t<RMAX, 1>(d, idx, nidx, st);
  if (rpt <= 2) return qr_right_t<RMAX, 2>(d, idx, nidx, st);
  return qr_right_t<RMAX, 4>(d, idx, nidx, st);
}

// Problems of one class (RMAX >= R_s, RPT * 512 >= n_s R_{s+1}, at most 4
// rows per thread) in one launch.
hipError_t launch_qr_right_batched(const BRo* d, const int32_t* idx, int32_t nidx, int32_t rmax, int32_t rpt,
                                   hipStream_t st) {
  if (nidx <= 0) return hipSuccess;
  if (rpt > 4) return hipErrorInvalidValue;
  if (rmax <= 4) return qr_right_r<4>(d, idx, nidx, rpt, st);
  if (rmax <= 8) return qr_right_r<8>(d, idx, nidx, rpt, st);
  if (rmax <= 12) return qr_right_r<12>(d, idx, nidx, rpt, st);
  return qr_right_r<16>(d, idx, nidx, rpt, st);
}

hipError_t launch_absorb_right_batched(const BRo* d, int32_t nprob, int32_t max_rows, hipStream_t st) {
  if (nprob <= 0 || max_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_absorb_right, dim3(nblk(max_rows, 256), (unsigned)nprob), dim3(256), 0, st, d);
  return hipGetLastError();
}
