// FP64 proximal solve (Sec. 3, (ite)).
//
// Solve: the split-K Gram partials of [SH^T SH | SH^T Y] are summed in FP64
// (k_gram_sum); M = SH^T SH + lambda I is factored M = L L^T by a blocked
// right-looking Cholesky (packed lower triangle in LDS, one workgroup); a
// second kernel forms B = SH^T Y + lambda G_(2)^T for a block of columns and
// solves L L^T Z = B by blocked forward and back substitution in LDS, one
// workgroup per block of columns.
// lambda > 0 makes M positive definite (Sec. 3, remark after (ite)); a
// non-positive pivot records TT_ERR_NOT_SPD in the status word.
//
// Blocks of 16 pivots.  The critical path is the chain of pivots, so it is
// kept short:
//  * the 16 x 16 diagonal block is factored in the registers of one wave
//    (lane (i, q) holds row i, columns q, q+4, q+8, q+12), pivots taken with
//    readlane and column values broadcast with shuffles, and 1/sqrt(d) is the
//    hardware estimate refined by two Newton steps (sqrt(d) = d / sqrt(d));
//  * the panel below it is solved one row per thread against a dense
//    transposed copy of the block and its reciprocal pivots, and 16 more
//    threads invert the block the same way (W_b = L_b^-1, stored after the
//    packed triangle), so the substitution's diagonal steps are products;
//  * the trailing updates (the Cholesky's lower triangle, the substitutions'
//    remaining rows) are 16 x 16 tiles of FP64 MFMA (v_mfma_f64_16x16x4f64)
//    over the block's 16 columns, operands read straight from LDS.
#include "tt_internal.h"

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kBS = 16;                         // pivots per block
constexpr int kLbLd = kBS + 1;                  // leading dimension of the dense block copy
constexpr int kCholExtra = kBS * kLbLd + kBS;   // doubles after the packed triangle

// Column-major packed lower triangle: column c holds rows c..s-1.
__device__ __forceinline__ int coff(int c, int s) { return c * s - (c * (c - 1)) / 2; }
__device__ __forceinline__ int lidx(int i, int c, int s) { return coff(c, s) + (i - c); }   // i >= c

// x of lane l (l the same in every lane)
__device__ __forceinline__ double lane_value(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}

// 1/sqrt(d) for finite d > 0: the hardware estimate and two Newton steps
// y <- y (3 - d y^2) / 2 (each step roughly doubles the correct bits).
__device__ __forceinline__ double rsqrt_newton(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double hd = 0.5 * d;
  y = y * (1.5 - hd * y * y);
  y = y * (1.5 - hd * y * y);
  return y;
}

__device__ __forceinline__ doublex4 mfma16(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// M (row i at M + i ldg, the lower triangle read) + lambda I = L L^T; L
// packed to Lout, followed by W_b = L_b^-1 of each 16 x 16 diagonal block
// (column-major, 256 doubles per block).  LDS: the packed triangle, then the dense copy of the
// current diagonal block (LbT[c kLbLd + i] = L[j0 + i][j0 + c]) and its
// reciprocal pivots.
__device__ __forceinline__ void chol_blk_body(cgdbl __restrict__ M, int32_t s, int32_t ldg, double lambda,
                                              gdbl __restrict__ Lout, int32_t* __restrict__ status, double* L,
                                              int& bad) {
  const int tid = threadIdx.x, T = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, NW = T >> 6;
  const int np = s * (s + 1) / 2;
  double* LbT = L + np;
  double* rinv = LbT + kBS * kLbLd;
  if (tid == 0) bad = 0;
  // a wave per row (contiguous in c), four rows in flight
  for (int i0 = wv; i0 < s; i0 += 4 * NW) {
    double v[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        const int i = i0 + q * NW, c = lane + 64 * h;
        v[q][h] = (i < s && c <= i) ? M[(int64_t)i * ldg + c] : 0.0;
      }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        const int i = i0 + q * NW, c = lane + 64 * h;
        if (i < s && c <= i) L[lidx(i, c, s)] = v[q][h] + (i == c ? lambda : 0.0);
      }
  }
  __syncthreads();
  for (int j0 = 0; j0 < s; j0 += kBS) {
    const int bs = min(kBS, s - j0), j1 = j0 + bs;
    // (a) diagonal block in the registers of wave 0; rows and columns beyond
    // the matrix are padded with the identity
    if (wv == 0) {
      const int i = lane & 15, q = lane >> 4;
      double a[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = q + 4 * k;
        a[k] = (i < bs && c <= i) ? L[lidx(j0 + i, j0 + c, s)] : (i == c ? 1.0 : 0.0);
      }
      bool ok = true;
#pragma unroll
      for (int p = 0; p < kBS; ++p) {
        const int src = p + 16 * (p & 3);   // lane holding A[p][p], slot p / 4
        const double d = lane_value(a[p >> 2], src);
        const bool good = d > 0.0 && isfinite(d);
        ok = ok && good;
        const double y = good ? rsqrt_newton(d) : 0.0;
        if (q == (p & 3)) {
          if (i == p) a[p >> 2] = d * y;
          else if (i > p) a[p >> 2] *= y;
        }
        if (lane == 0) rinv[p] = y;
        const double li = __shfl(a[p >> 2], i + 16 * (p & 3), 64);   // L[i][p]
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int c = q + 4 * k;
          const double lc = __shfl(a[p >> 2], c + 16 * (p & 3), 64);   // L[c][p]
          if (c > p && c <= i) a[k] -= li * lc;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = q + 4 * k;
        if (i < bs && c <= i) L[lidx(j0 + i, j0 + c, s)] = a[k];
        if (c < i) LbT[c * kLbLd + i] = a[k];   // zero in the padding rows
      }
      if (lane == 0 && !ok) bad = 1;
    }
    __syncthreads();
    if (bad) break;
    // (b) panel rows i >= j1: L[i][j0:j1] <- M[i][j0:j1] L_blk^-T (a forward
    // substitution per row).  Meanwhile the last 16 threads run the same
    // substitution on unit vectors: W_b = L_blk^-1, stored column-major
    // after the packed triangle for the substitution kernel.  Padding
    // columns stay zero (rinv = 1, zero couplings), so the loops need no
    // bounds and every load can be issued early.
    for (int i = j1 + tid; i < s; i += T) {
      double x[kBS];
#pragma unroll
      for (int u = 0; u < kBS; ++u) {
        const double t = L[lidx(i, j0 + min(u, bs - 1), s)];
        x[u] = u < bs ? t : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kBS; ++u) {
        x[u] *= rinv[u];
#pragma unroll
        for (int v = u + 1; v < kBS; ++v) x[v] -= LbT[u * kLbLd + v] * x[u];
      }
#pragma unroll
      for (int u = 0; u < kBS; ++u)
        if (u < bs) L[lidx(i, j0 + u, s)] = x[u];
    }
    if (tid >= T - kBS) {   // s <= TT_MAX_S keeps these threads out of the panel
      const int c = tid - (T - kBS);
      double x[kBS];
#pragma unroll
      for (int u = 0; u < kBS; ++u) x[u] = u == c ? 1.0 : 0.0;
#pragma unroll
      for (int u = 0; u < kBS; ++u) {
        x[u] *= rinv[u];
#pragma unroll
        for (int v = u + 1; v < kBS; ++v) x[v] -= LbT[u * kLbLd + v] * x[u];
      }
      const gdbl W = Lout + np + (size_t)(j0 / kBS) * kBS * kBS;
#pragma unroll
      for (int u = 0; u < kBS; ++u) W[u + kBS * c] = x[u];   // W[u][c]
    }
    __syncthreads();
    // (c) trailing update A22 -= L21 L21^T, lower 16 x 16 tiles, a wave per tile
    const int R = s - j1;
    if (R > 0) {
      const int nt = (R + 15) / 16;
      const int rl = lane & 15, kq = lane >> 4;
      int e = 0;
      for (int ti = 0; ti < nt; ++ti)
        for (int tc = 0; tc <= ti; ++tc, ++e) {
          if (e % NW != wv) continue;
          const int i0 = j1 + 16 * ti, c0 = j1 + 16 * tc;
          doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kk = 0; kk < kBS; kk += 4) {
            const int u = kk + kq, uc = j0 + min(u, bs - 1);
            const int ia = i0 + rl, ic = c0 + rl;
            const double ta = L[lidx(min(ia, s - 1), uc, s)], tb = L[lidx(min(ic, s - 1), uc, s)];
            const double av = (u < bs && ia < s) ? ta : 0.0;
            const double bv = (u < bs && ic < s) ? tb : 0.0;
            acc = mfma16(av, bv, acc);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {   // D[row 4 r + kq][col rl]
            const int row = i0 + 4 * r + kq, col = c0 + rl;
            if (row < s && col <= row) L[lidx(row, col, s)] -= acc[r];
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

__global__ __launch_bounds__(256) void k_chol_blk(const double* __restrict__ M, int32_t s, int32_t ldg, double lambda,
                                                 double* __restrict__ Lout, int32_t* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int bad;
  chol_blk_body((cgdbl)M, s, ldg, lambda, (gdbl)Lout, status, reinterpret_cast<double*>(smem_raw), bad);
}

// Columns c0 .. c0 + CB - 1 (CB a power of two) of
// B = (SH^T Y)(:, cols) + lambda G_(2)^T, the right-hand side (row j of M + j
// ldg, columns s..), solved in place by L y = B (forward) and L^T z = y
// (backward), 16 rows at a time.  The diagonal step of a block is a product
// with the block's inverse W_b (written by the Cholesky kernel after the
// packed triangle): y_b = W_b B_b forward, z_b = W_b^T y_b backward; then all
// waves update the rows the block feeds.  Both are 16 x 16 MFMA tiles.  LDS:
// L (packed) and B (s x CB, row-major); W_b is read from L2.
__device__ __forceinline__ void trsm_blk_body(cgdbl __restrict__ M, int32_t s, int32_t ldg, double lambda,
                                              cgdbl __restrict__ Lg, cgdbl G_old, gdbl G_new, int32_t rk, int32_t nk,
                                              int32_t CB, int bx, double* L) {
  const int np = s * (s + 1) / 2;
  double* Bs = L + np;
  const cgdbl Wg = Lg + np;
  const int c0 = bx * CB;
  const int lcb = __builtin_ctz((unsigned)CB);
  const int tid = threadIdx.x, T = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, NW = T >> 6;
  const int rl = lane & 15, kq = lane >> 4;
  // loads four per thread in flight
  for (int e0 = tid; e0 < np; e0 += 4 * T) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = e0 + q * T < np ? Lg[e0 + q * T] : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (e0 + q * T < np) L[e0 + q * T] = v[q];
  }
  for (int e0 = tid; e0 < s * CB; e0 += 4 * T) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = e0 + q * T;
      const int j = e >> lcb, col = c0 + (e & (CB - 1));
      v[q] = 0.0;
      if (e < s * CB && col < nk) {
        const int a = j % rk, b = j / rk;
        v[q] = M[(int64_t)j * ldg + s + col] + lambda * G_old[a + (int64_t)rk * (col + (int64_t)nk * b)];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (e0 + q * T < s * CB) Bs[e0 + q * T] = v[q];
  }
  __syncthreads();   // every read of G_old for these columns precedes the writes below
  const int ctiles = (CB + 15) / 16;
  // forward: L y = B
  for (int j0 = 0; j0 < s; j0 += kBS) {
    const int bs = min(kBS, s - j0), j1 = j0 + bs;
    const cgdbl Wb = Wg + (size_t)(j0 / kBS) * kBS * kBS;
    for (int t = wv; t < ctiles; t += NW) {   // y_b = W_b B_b, a wave per column tile
      const int cc = 16 * t;
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < kBS; kk += 4) {
        const int u = kk + kq, cb = cc + rl;
        const double av = Wb[rl + kBS * u];   // W[rl][u]
        const double tb = Bs[min(j0 + u, s - 1) * CB + min(cb, CB - 1)];
        acc = mfma16(av, (u < bs && cb < CB) ? tb : 0.0, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = j0 + 4 * r + kq, col = cc + rl;
        if (row < s && col < CB) Bs[row * CB + col] = acc[r];
      }
    }
    __syncthreads();
    // rows i >= j1: B[i][:] -= L[i][j0:j1] y[j0:j1][:]
    const int rtiles = (s - j1 + 15) / 16;
    for (int t = wv; t < rtiles * ctiles; t += NW) {
      const int i0 = j1 + 16 * (t / ctiles), cc = 16 * (t % ctiles);
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < kBS; kk += 4) {
        const int u = kk + kq, uc = j0 + min(u, bs - 1);
        const int ia = i0 + rl, cb = cc + rl;
        const double ta = L[lidx(min(ia, s - 1), uc, s)], tb = Bs[uc * CB + min(cb, CB - 1)];
        const double av = (u < bs && ia < s) ? ta : 0.0;
        const double bv = (u < bs && cb < CB) ? tb : 0.0;
        acc = mfma16(av, bv, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + 4 * r + kq, col = cc + rl;
        if (row < s && col < CB) Bs[row * CB + col] -= acc[r];
      }
    }
    __syncthreads();
  }
  // backward: L^T z = y
  for (int j0 = ((s - 1) / kBS) * kBS; j0 >= 0; j0 -= kBS) {
    const int bs = min(kBS, s - j0);
    const cgdbl Wb = Wg + (size_t)(j0 / kBS) * kBS * kBS;
    for (int t = wv; t < ctiles; t += NW) {   // z_b = W_b^T y_b
      const int cc = 16 * t;
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < kBS; kk += 4) {
        const int u = kk + kq, cb = cc + rl;
        const double av = Wb[u + kBS * rl];   // W[u][rl]
        const double tb = Bs[min(j0 + u, s - 1) * CB + min(cb, CB - 1)];
        acc = mfma16(av, (u < bs && cb < CB) ? tb : 0.0, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = j0 + 4 * r + kq, col = cc + rl;
        if (row < s && col < CB) Bs[row * CB + col] = acc[r];
      }
    }
    __syncthreads();
    // rows i < j0: B[i][:] -= sum_u L[j0 + u][i] z[j0 + u][:]
    const int rtiles = j0 / 16;
    for (int t = wv; t < rtiles * ctiles; t += NW) {
      const int i0 = 16 * (t / ctiles), cc = 16 * (t % ctiles);
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < kBS; kk += 4) {
        const int u = kk + kq, uc = j0 + min(u, bs - 1);
        const int cb = cc + rl;
        const double ta = L[lidx(uc, i0 + rl, s)], tb = Bs[uc * CB + min(cb, CB - 1)];
        const double av = u < bs ? ta : 0.0;
        const double bv = (u < bs && cb < CB) ? tb : 0.0;
        acc = mfma16(av, bv, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + 4 * r + kq, col = cc + rl;
        if (col < CB) Bs[row * CB + col] -= acc[r];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < s * CB; e += T) {
    const int q = e >> lcb, col = c0 + (e & (CB - 1));
    if (col < nk) {
      const int a = q % rk, b = q / rk;
      G_new[a + (int64_t)rk * (col + (int64_t)nk * b)] = Bs[e];
    }
  }
}

__global__ __launch_bounds__(256) void k_prox_trsm_blk(const double* __restrict__ M, int32_t s, int32_t ldg,
                                                      double lambda, const double* __restrict__ Lg,
                                                      const double* G_old, double* G_new, int32_t rk, int32_t nk,
                                                      int32_t CB) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  trsm_blk_body((cgdbl)M, s, ldg, lambda, (cgdbl)Lg, (cgdbl)G_old, (gdbl)G_new, rk, nk, CB, blockIdx.x,
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
  chol_blk_body((cgdbl)u.gsum, u.s, u.s + u.nk, u.lambda, (gdbl)u.Lg, u.status, reinterpret_cast<double*>(smem_raw),
                bad);
}

__global__ __launch_bounds__(256) void kb_trsm(const BUpd* __restrict__ d) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const BUpd u = d[blockIdx.y];
  if ((int)blockIdx.x * u.CB >= u.nk) return;
  trsm_blk_body((cgdbl)u.gsum, u.s, u.s + u.nk, u.lambda, (cgdbl)u.Lg, (cgdbl)u.G, (gdbl)u.G, u.rk, u.nk, u.CB, blockIdx.x,
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

// Cholesky of gsum's s x s block plus lambda I and the blocked substitution
// of its n_k right-hand-side columns plus lambda G_(2)^T; gsum is row-major
// s x (s + n_k) in the plan's o_gsum buffer.
hipError_t solve_from_gsum(const tt_plan_s* p, int k, const double* G_old, double* G_new) {
  const int s = (int)(p->r[k] * p->r[k + 1]);
  const int nk = (int)p->n[k];
  const int ldg = s + nk;
  double* Lg = p->at<double>(p->o_minv);
  int32_t* status = p->at<int32_t>(p->o_status);
  const double* gsum = p->at<double>(p->o_gsum);
  hipError_t e;
  const size_t np = (size_t)s * (s + 1) / 2;
  const size_t lds1 = tt_chol_lds_bytes(s);
  if ((e = tt_allow_lds(k_chol_blk, lds1)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_blk, dim3(1), dim3(256), lds1, p->stream, gsum, s, ldg, p->lambda, Lg, status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // right-hand-side block of 8 columns (a 16-wide MFMA tile half used): each
  // workgroup's time is the latency of its 2 ceil(s / 16) block steps, not
  // their MFMA work, so narrow blocks and more workgroups finish first
  // (s = 100, n = 200: 56 / 38 / 28 / 27 us at 64 / 32 / 16 / 8 columns);
  // narrower still if L and the block do not fit in 150 KB of LDS
  int CB = 8;
  while (CB > 1 && (np + (size_t)s * CB) * sizeof(double) > 150 * 1024) CB >>= 1;
  const size_t lds2 = (np + (size_t)s * CB) * sizeof(double);
  if ((e = tt_allow_lds(k_prox_trsm_blk, lds2)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_prox_trsm_blk, dim3(nblk(nk, CB)), dim3(256), lds2, p->stream, gsum, s, ldg,
                     p->lambda, Lg, G_old, G_new, (int32_t)p->r[k], nk, CB);
  return hipGetLastError();
}

template <typename AT>
hipError_t prox_t(const tt_plan_s* p, int k, const double* G_old, double* G_new) {
  const int s = (int)(p->r[k] * p->r[k + 1]);
  const int nk = (int)p->n[k];
  const int ldg = s + nk;
  const int chunks = (int)tt_gram_chunks(p->J);
  // the split-K partials summed once, every entry in parallel; the solve
  // kernels then read one FP64 copy
  double* gsum = p->at<double>(p->o_gsum);
  const int64_t count = (int64_t)s * ldg;
  hipLaunchKernelGGL(k_gram_sum<AT>, dim3(nblk(count, 256)), dim3(256), 0, p->stream, p->at<AT>(p->o_gram), chunks,
                     count, gsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return solve_from_gsum(p, k, G_old, G_new);
}

}  // namespace

size_t tt_chol_lds_bytes(int64_t s) { return (size_t)(s * (s + 1) / 2 + kCholExtra) * sizeof(double); }
int64_t tt_chol_out_doubles(int64_t s) { return s * (s + 1) / 2 + ((s + kBS - 1) / kBS) * kBS * kBS; }

hipError_t launch_prox_from_gsum(const tt_plan_s* p, int k, const double* G_old, double* G_new) {
  return solve_from_gsum(p, k, G_old, G_new);
}

hipError_t launch_prox_from_gram(const tt_plan_s* p, int k, const double* G_old, double* G_new) {
  // FP32 partials only under TT_GRAM_BF16 (FP32 MFMA accumulation)
  return p->gram_mode == TT_GRAM_BF16 ? prox_t<float>(p, k, G_old, G_new) : prox_t<double>(p, k, G_old, G_new);
}

hipError_t launch_copy_f64(const tt_plan_s* p, double* dst, const double* src, int64_t count) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f64, dim3(nblk(count, 256)), dim3(256), 0, p->stream, dst, src, count);
  return hipGetLastError();
}

hipError_t launch_gram_sum_batched(const BUpd* d, int32_t nprob, int32_t max_count, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_gram_sum, dim3(nblk(max_count, 256), (unsigned)nprob), dim3(256), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_solve_batched(const BUpd* d, int32_t nprob, int32_t max_s, int32_t max_count, int32_t max_cb_blocks,
                                size_t lds_chol, size_t lds_trsm, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  (void)max_s;
  hipError_t e = launch_gram_sum_batched(d, nprob, max_count, st);
  if (e != hipSuccess) return e;
  if ((e = tt_allow_lds(kb_chol, lds_chol)) != hipSuccess) return e;
  hipLaunchKernelGGL(kb_chol, dim3((unsigned)nprob), dim3(256), lds_chol, st, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = tt_allow_lds(kb_trsm, lds_trsm)) != hipSuccess) return e;
  hipLaunchKernelGGL(kb_trsm, dim3((unsigned)max_cb_blocks, (unsigned)nprob), dim3(256), lds_trsm, st, d);
  return hipGetLastError();
}
