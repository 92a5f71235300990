// FP64 proximal solve (Sec. 3, eq. (3.5)) and the QR steps of Algorithm 1.
//
// Solve: M = SH^T SH + lambda I is summed from the Gram partials in FP64,
// factored M = L L^T (Cholesky, packed lower triangle in LDS), L is inverted
// in place and M^{-1} = L^{-T} L^{-1} is formed; a second kernel applies
// M^{-1} to B = SH^T Y + lambda G_(2)^T, one workgroup per block of columns.
// lambda > 0 makes M positive definite (Sec. 3, remark after eq. (3.5)); a
// non-positive pivot records TT_ERR_NOT_SPD in the status word.
//
// QR: Householder QR of a tall m x r FP64 operand (one workgroup), with the
// LAPACK reflector convention (tau = 0 when the column below the diagonal is
// zero), the explicit Q accumulated backwards, and the sign normalisation
// diag(R) >= 0.  The operand is read and Q written back through (row, col)
// strides so one kernel serves both G_k^L (left-orthogonalisation) and
// (G_k^R)^T (right-to-left orthogonalisation).
#include "tt_internal.h"

namespace {

constexpr int kSolveThreads = 1024;

__device__ __forceinline__ int pidx(int i, int j) { return i * (i + 1) / 2 + j; }  // i >= j

template <typename AT>
__global__ __launch_bounds__(kSolveThreads) void k_chol_inv(const AT* __restrict__ gpart, int32_t chunks, int32_t s,
                                                           int32_t ldg, double lambda, double* __restrict__ Minv,
                                                           int32_t* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* L = reinterpret_cast<double*>(smem_raw);             // packed lower, s(s+1)/2
  double* tmp = L + s * (s + 1) / 2;                           // s
  __shared__ int bad;
  const int tid = threadIdx.x, T = blockDim.x;
  const int np = s * (s + 1) / 2;
  if (tid == 0) bad = 0;
  for (int e = tid; e < np; e += T) {
    // decode packed index e -> (i, j), i >= j
    int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (pidx(i + 1, 0) <= e) ++i;
    while (pidx(i, 0) > e) --i;
    const int j = e - pidx(i, 0);
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += (double)gpart[((int64_t)c * s + i) * ldg + j];
    L[e] = acc + (i == j ? lambda : 0.0);
  }
  __syncthreads();
  // right-looking Cholesky
  for (int j = 0; j < s; ++j) {
    const double djj = L[pidx(j, j)];
    if (!(djj > 0.0) || !isfinite(djj)) {
      if (tid == 0) bad = 1;
      break;   // uniform: every thread read the same pivot
    }
    const double dj = sqrt(djj);
    __syncthreads();
    for (int i = j + 1 + tid; i < s; i += T) L[pidx(i, j)] /= dj;
    if (tid == 0) L[pidx(j, j)] = dj;
    __syncthreads();
    // trailing update of the packed lower triangle rows i > j, columns j < c <= i
    const int m = s - j - 1;
    const int nt = m * (m + 1) / 2;
    for (int e = tid; e < nt; e += T) {
      int ii = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
      while (ii * (ii + 1) / 2 > e) --ii;
      const int cc = e - ii * (ii + 1) / 2;
      const int i = j + 1 + ii, c = j + 1 + cc;
      L[pidx(i, c)] -= L[pidx(i, j)] * L[pidx(c, j)];
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    for (int e = tid; e < s * s; e += T) Minv[e] = __longlong_as_double(0x7ff8000000000000ll);
    if (tid == 0) atomicOr(status, 1);
    return;
  }
  // in-place inverse of the lower triangle (unblocked, from the bottom right)
  for (int j = s - 1; j >= 0; --j) {
    if (tid == 0) L[pidx(j, j)] = 1.0 / L[pidx(j, j)];
    __syncthreads();
    const double ajj = -L[pidx(j, j)];
    // x = L[j+1:, j];  x <- T x with T = inverted trailing block (lower)
    for (int i = j + 1 + tid; i < s; i += T) {
      double acc = 0.0;
      for (int m = j + 1; m <= i; ++m) acc += L[pidx(i, m)] * L[pidx(m, j)];
      tmp[i] = acc * ajj;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < s; i += T) L[pidx(i, j)] = tmp[i];
    __syncthreads();
  }
  // M^{-1} = W^T W with W = L^{-1} (lower): (W^T W)_{ij} = sum_{m >= max(i,j)} W_mi W_mj
  for (int e = tid; e < s * s; e += T) {
    const int i = e / s, j = e - (e / s) * s;
    const int lo = i > j ? i : j;
    double acc = 0.0;
    for (int m = lo; m < s; ++m) acc += L[pidx(m, i)] * L[pidx(m, j)];
    Minv[e] = acc;
  }
}

// G_new(a, col, b) = sum_j Minv[q][j] B[j][col], q = a + R_k b,
// B[j][col] = sum_c gpart[c][j][s + col] + lambda G_old(a_j, col, b_j).
template <typename AT, int CB>
__global__ __launch_bounds__(256) void k_prox_apply(const AT* __restrict__ gpart, int32_t chunks, int32_t s, int32_t ldg,
                                                   double lambda, const double* __restrict__ Minv, const double* G_old,
                                                   double* G_new, int32_t rk, int32_t nk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Bs = reinterpret_cast<double*>(smem_raw);   // s x CB, col fastest
  const int c0 = blockIdx.x * CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < s * CB; e += blockDim.x) {
    const int j = e / CB, cl = e - (e / CB) * CB;
    const int col = c0 + cl;
    double acc = 0.0;
    if (col < nk) {
      for (int c = 0; c < chunks; ++c) acc += (double)gpart[((int64_t)c * s + j) * ldg + s + col];
      const int a = j % rk, b = j / rk;
      acc += lambda * G_old[a + (int64_t)rk * (col + (int64_t)nk * b)];
    }
    Bs[e] = acc;
  }
  __syncthreads();   // every read of G_old for these columns precedes the writes below
  for (int e = tid; e < s * CB; e += blockDim.x) {
    const int q = e / CB, cl = e - (e / CB) * CB;
    const int col = c0 + cl;
    if (col >= nk) continue;
    const double* mrow = Minv + (int64_t)q * s;
    double acc = 0.0;
    for (int j = 0; j < s; ++j) acc += mrow[j] * Bs[j * CB + cl];
    const int a = q % rk, b = q / rk;
    G_new[a + (int64_t)rk * (col + (int64_t)nk * b)] = acc;
  }
}

// ---------------------------------------------------------------- QR
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
  const AT* gpart = p->at<AT>(p->o_gram);
  double* Minv = p->at<double>(p->o_minv);
  int32_t* status = p->at<int32_t>(p->o_status);
  const size_t lds1 = ((size_t)s * (s + 1) / 2 + s) * sizeof(double);
  hipError_t e0 = tt_allow_lds(k_chol_inv<AT>, lds1);
  if (e0 != hipSuccess) return e0;
  hipLaunchKernelGGL(k_chol_inv<AT>, dim3(1), dim3(kSolveThreads), lds1, p->stream, gpart, chunks, s, ldg, p->lambda,
                     Minv, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int CB = 32;
  const size_t lds2 = (size_t)s * CB * sizeof(double);
  hipLaunchKernelGGL((k_prox_apply<AT, CB>), dim3(nblk(nk, CB)), dim3(256), lds2, p->stream, gpart, chunks, s, ldg,
                     p->lambda, Minv, G_old, G_new, (int32_t)p->r[k], nk);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_prox_from_gram(const tt_plan_s* p, int k, const double* G_old, double* G_new) {
  return p->wdt == TT_F64 ? prox_t<double>(p, k, G_old, G_new) : prox_t<float>(p, k, G_old, G_new);
}

hipError_t launch_qr_core(const tt_plan_s* p, double* G, int64_t m, int64_t rcols, int64_t rs, int64_t cs) {
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

hipError_t launch_copy_f64(const tt_plan_s* p, double* dst, const double* src, int64_t count) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f64, dim3(nblk(count, 256)), dim3(256), 0, p->stream, dst, src, count);
  return hipGetLastError();
}
