// FP64 proximal solve (Sec. 3, eq. (3.5)).
//
// Solve: M = SH^T SH + lambda I is summed from the Gram partials in FP64 and
// factored M = L L^T (right-looking Cholesky, packed lower triangle in LDS,
// one workgroup); a second kernel forms B = SH^T Y + lambda G_(2)^T for a
// block of columns and solves L L^T Z = B by forward and back substitution in
// LDS, one workgroup per block of columns.
// lambda > 0 makes M positive definite (Sec. 3, remark after eq. (3.5)); a
// non-positive pivot records TT_ERR_NOT_SPD in the status word.
#include "tt_internal.h"

namespace {

constexpr int kSolveThreads = 1024;

// Column-major packed lower triangle: column c holds rows c..s-1.
__device__ __forceinline__ int coff(int c, int s) { return c * s - (c * (c - 1)) / 2; }
__device__ __forceinline__ int lidx(int i, int c, int s) { return coff(c, s) + (i - c); }   // i >= c

// M = sum of the Gram partials + lambda I (lower triangle), factored
// M = L L^T in LDS; L is written (packed) to Lout.  One workgroup.
template <typename AT>
__global__ __launch_bounds__(kSolveThreads) void k_chol(const AT* __restrict__ gpart, int32_t chunks, int32_t s,
                                                       int32_t ldg, double lambda, double* __restrict__ Lout,
                                                       int32_t* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* L = reinterpret_cast<double*>(smem_raw);
  __shared__ int bad;
  const int tid = threadIdx.x, T = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, NW = T >> 6;
  const int np = s * (s + 1) / 2;
  if (tid == 0) bad = 0;
  for (int c = wv; c < s; c += NW)
    for (int i = c + lane; i < s; i += 64) {
      double acc = 0.0;
      for (int q = 0; q < chunks; ++q) acc += (double)gpart[((int64_t)q * s + i) * ldg + c];
      L[lidx(i, c, s)] = acc + (i == c ? lambda : 0.0);
    }
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    const double djj = L[lidx(j, j, s)];
    if (!(djj > 0.0) || !isfinite(djj)) {
      if (tid == 0) bad = 1;
      break;   // uniform: every thread read the same pivot
    }
    const double dj = sqrt(djj);
    const double inv = 1.0 / dj;
    __syncthreads();   // all threads have read the pivot before it is overwritten
    for (int i = j + 1 + tid; i < s; i += T) L[lidx(i, j, s)] *= inv;
    if (tid == 0) L[lidx(j, j, s)] = dj;
    __syncthreads();
    for (int c = j + 1 + wv; c < s; c += NW) {
      const double lcj = L[lidx(c, j, s)];
      const int oc = coff(c, s) - c, oj = coff(j, s) - j;
      for (int i = c + lane; i < s; i += 64) L[oc + i] -= L[oj + i] * lcj;
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    for (int e = tid; e < np; e += T) Lout[e] = __longlong_as_double(0x7ff8000000000000ll);
    if (tid == 0) atomicOr(status, 1);
    return;
  }
  for (int e = tid; e < np; e += T) Lout[e] = L[e];
}

// For a block of CB right-hand-side columns: B = SH^T Y + lambda G_(2)^T (from
// the Gram partials), then L y = B and L^T z = y by column-oriented
// substitution in LDS (one barrier per pivot; row normalisation deferred),
// and z is stored as the new core columns.
template <typename AT>
__global__ __launch_bounds__(256) void k_prox_trsm(const AT* __restrict__ gpart, int32_t chunks, int32_t s, int32_t ldg,
                                                  double lambda, const double* __restrict__ Lg, const double* G_old,
                                                  double* G_new, int32_t rk, int32_t nk, int32_t CB) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int np = s * (s + 1) / 2;
  double* L = reinterpret_cast<double*>(smem_raw);
  double* Bs = L + np;                 // s x CB, column block index fastest
  double* invd = Bs + (size_t)s * CB;  // s
  const int c0 = blockIdx.x * CB;
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
  // forward: rows i > j take row j (final, not yet scaled) times L(i,j)/L(j,j)
  for (int j = 0; j < s - 1; ++j) {
    const double dj = invd[j];
    const int oj = coff(j, s) - j;
    const int n = (s - 1 - j) * CB;
    for (int e = tid; e < n; e += T) {
      const int ii = e / CB, cl = e - ii * CB;
      const int i = j + 1 + ii;
      Bs[i * CB + cl] -= L[oj + i] * dj * Bs[j * CB + cl];
    }
    __syncthreads();
  }
  for (int e = tid; e < s * CB; e += T) Bs[e] *= invd[e / CB];
  __syncthreads();
  // backward: L^T z = y, rows i < j take z_j = row j / L(j,j) times L(j,i)
  for (int j = s - 1; j > 0; --j) {
    const double dj = invd[j];
    const int n = j * CB;
    for (int e = tid; e < n; e += T) {
      const int i = e / CB, cl = e - i * CB;
      Bs[i * CB + cl] -= L[lidx(j, i, s)] * dj * Bs[j * CB + cl];
    }
    __syncthreads();
  }
  for (int e = tid; e < s * CB; e += T) {
    const int q = e / CB, cl = e - q * CB;
    const int col = c0 + cl;
    if (col < nk) {
      const int a = q % rk, b = q / rk;
      G_new[a + (int64_t)rk * (col + (int64_t)nk * b)] = Bs[e] * invd[q];
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
  double* Lg = p->at<double>(p->o_minv);
  int32_t* status = p->at<int32_t>(p->o_status);
  const size_t np = (size_t)s * (s + 1) / 2;
  const size_t lds1 = np * sizeof(double);
  hipError_t e = tt_allow_lds(k_chol<AT>, lds1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol<AT>, dim3(1), dim3(kSolveThreads), lds1, p->stream, gpart, chunks, s, ldg, p->lambda, Lg,
                     status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // right-hand-side block: as wide as fits next to L in 150 KB of LDS
  int CB = 64;
  while (CB > 1 && (np + (size_t)s * CB + s) * sizeof(double) > 150 * 1024) CB >>= 1;
  const size_t lds2 = (np + (size_t)s * CB + s) * sizeof(double);
  if ((e = tt_allow_lds(k_prox_trsm<AT>, lds2)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_prox_trsm<AT>, dim3(nblk(nk, CB)), dim3(256), lds2, p->stream, gpart, chunks, s, ldg, p->lambda,
                     Lg, G_old, G_new, (int32_t)p->r[k], nk, CB);
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
