// Exact (unsketched) proximal update of core k, the subproblem
// (lrtt_sub_prox) of Sec. 3, solved in closed form:
//   G_k(2)^new = (A_(k) H_k + lambda G_k(2)^old) (H_k^T H_k + lambda I)^{-1},
//   H_k = G_{>k}^T (x) G_{<k}.
// A_(k) H_k is never formed through H_k.  X is contracted with the cores one
// mode at a time, which keeps every intermediate at most R N / n_i values:
//  * left interface Phi_k = X contracted over modes 0..k-1 with G_0..G_{k-1},
//    shape (R_k, n_k, ..., n_{d-1}); Phi_0 = X and Phi_{k+1} = Phi_k
//    contracted over (alpha, i_k) with G_k (k_contract_fast: the contracted
//    index is the contiguous one, so each column is a dot product with a
//    column of G_k; FP64 MFMA does the reduction);
//  * right chain: Phi_k contracted over modes d-1, d-2, ..., k+1 with their
//    cores (k_contract_slow: the contracted index is the slowest one, lanes
//    run along the contiguous index, one FP64 FMA per entry and rank), which
//    ends at B_k(alpha, i_k, beta) = (A_(k) H_k)(i_k, alpha + R_k beta).
// H_k^T H_k = (G_{>k} G_{>k}^T) (x) (G_{<k}^T G_{<k}) from two small Gram
// recursions (identity in the gauge of a sweep, where the cores left of k
// are left-orthonormal and those right of k right-orthonormal).  The FP64
// Cholesky and substitution are the sketched update's (k_solve.hip).
#include <math.h>

#include <vector>

#include "tt_internal.h"

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ double to_f64(T v) { return (double)v; }
template <>
__device__ __forceinline__ double to_f64<uint16_t>(uint16_t v) { return (double)__uint_as_float((uint32_t)v << 16); }

// 4 consecutive values of T (k .. k+3 of one column) in their storage type;
// zero beyond K
template <typename TT, bool VEC>
__device__ __forceinline__ void load4(const TT* __restrict__ col, int64_t k, int64_t K, TT (&v)[4]) {
  if constexpr (VEC) {
    typedef TT raw_t __attribute__((ext_vector_type(4)));
    if (k + 3 < K) {
      const raw_t r = *reinterpret_cast<const raw_t*>(col + k);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = r[e];
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = k + e < K ? col[k + e] : (TT)0;
}

// Out(b, q) = sum_{k < K} G[k + K b] T[k + K q] for b < Rout, q < Q, with the
// K range of slice blockIdx.y (K = R_in n, contiguous per column q; G is the
// core (R_in, n, R_out), i.e. a K x R_out column-major matrix).  One wave:
// NT tiles of 16 columns; v_mfma_f64_16x16x4f64 with A(row b, k) = G and
// B(k, column q) = T.  Lane l loads 4 consecutive k of column l % 16 at
// offset 4 (l / 16) of each 16-value step and feeds them to 4 MFMAs, so a
// column is read in 64-byte pieces (FP32).  The loads of the next step are
// issued before the MFMAs of the current one, and values stay in their
// storage type until the MFMA (registers: two load buffers and the
// accumulators).  Results: lane l, register r hold row 4 r + l / 16, column
// l % 16.  S == 1 writes OT directly, else FP64 partials
// part[(s Q + q) R_out + b].
template <typename TT, typename OT, int NT, bool VEC>
__global__ __launch_bounds__(256) void k_contract_fast(const TT* __restrict__ T, const double* __restrict__ G,
                                                       OT* __restrict__ out, double* __restrict__ part, int64_t Q,
                                                       int64_t K, int32_t Rout, int32_t S) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t q0 = wave * 16 * NT;
  if (q0 >= Q) return;
  // slice bounds on multiples of 16, so that every 4-value load stays aligned
  const int s = blockIdx.y;
  const int64_t kb0 = ((int64_t)s * K / S) & ~(int64_t)15;
  const int64_t kb1 = s + 1 == S ? K : (((int64_t)(s + 1) * K / S) & ~(int64_t)15);
  const int kq = lane >> 4, nl = lane & 15;
  const bool brow = nl < Rout;
  const double* Gcol = G + K * (brow ? nl : 0);
  const TT* cols[NT];
  bool qok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int64_t q = q0 + 16 * t + nl;
    qok[t] = q < Q;
    cols[t] = T + K * (qok[t] ? q : 0);
  }
  doublex4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  auto issue = [&](TT (&x)[NT][4], int64_t kb) {
    const int64_t k = kb + 4 * kq;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (qok[t]) {
        load4<TT, VEC>(cols[t], k, kb1, x[t]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) x[t][e] = (TT)0;
      }
    }
  };
  auto consume = [&](const TT (&x)[NT][4], int64_t kb) {
    const int64_t k = kb + 4 * kq;
    double a[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = (brow && k + e < kb1) ? Gcol[k + e] : 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e], to_f64<TT>(x[t][e]), acc[t], 0, 0, 0);
  };
  TT xa[NT][4], xb[NT][4];
  if (kb0 < kb1) issue(xa, kb0);
  for (int64_t kb = kb0; kb < kb1; kb += 32) {
    if (kb + 16 < kb1) issue(xb, kb + 16);
    consume(xa, kb);
    if (kb + 16 >= kb1) break;
    if (kb + 32 < kb1) issue(xa, kb + 32);
    consume(xb, kb + 16);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (!qok[t]) continue;
    const int64_t q = q0 + 16 * t + nl;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int b = 4 * r + kq;
      if (b >= Rout) continue;
      if (S == 1)
        out[b + (int64_t)Rout * q] = (OT)acc[t][r];
      else
        part[((int64_t)s * Q + q) * Rout + b] = acc[t][r];
    }
  }
}

// Out(m, a) = sum_{kk < n R_in} T[m + M kk] G[a + R_out kk] for a < R_out
// (contraction of the slowest mode and the trailing rank), with the kk range
// of slice blockIdx.y.  Lanes run along m (coalesced), U loads in flight per
// lane; the core values are the same for the whole wave.  RB bounds R_out.
// S == 1 writes OT directly, else FP64 partials part[(s R_out + a) M + m].
template <typename TT, typename OT, int RB>
__global__ __launch_bounds__(256) void k_contract_slow(const TT* __restrict__ T, const double* __restrict__ G,
                                                       OT* __restrict__ out, double* __restrict__ part, int64_t M,
                                                       int64_t KK, int32_t Rout, int32_t S) {
  constexpr int U = 16;
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int64_t k0 = (int64_t)s * KK / S, k1 = (int64_t)(s + 1) * KK / S;
  double acc[RB];
#pragma unroll
  for (int a = 0; a < RB; ++a) acc[a] = 0.0;
  if (m < M) {
    const TT* col = T + m;
    int64_t kk = k0;
    for (; kk + U <= k1; kk += U) {
      TT x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = col[M * (kk + u)];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double xv = to_f64<TT>(x[u]);
        const double* g = G + (int64_t)Rout * (kk + u);
#pragma unroll
        for (int a = 0; a < RB; ++a)
          if (a < Rout) acc[a] += xv * g[a];
      }
    }
    for (; kk < k1; ++kk) {
      const double x = to_f64<TT>(col[M * kk]);
      const double* g = G + (int64_t)Rout * kk;
#pragma unroll
      for (int a = 0; a < RB; ++a)
        if (a < Rout) acc[a] += x * g[a];
    }
#pragma unroll
    for (int a = 0; a < RB; ++a) {
      if (a >= Rout) break;
      if (S == 1)
        out[m + M * a] = (OT)acc[a];
      else
        part[((int64_t)s * Rout + a) * M + m] = acc[a];
    }
  }
}

// The contraction of k_contract_slow for a long kk range (the two slow modes
// merged, KK = n_a n_b): the core rows of the slice are staged through LDS,
// CH at a time, so that the waves of a workgroup read them from LDS instead
// of each streaming the whole slice of the core from L2.
template <typename TT, typename OT, int RB>
__global__ __launch_bounds__(256) void k_contract_merged(const TT* __restrict__ T, const double* __restrict__ G,
                                                         OT* __restrict__ out, double* __restrict__ part, int64_t M,
                                                         int64_t KK, int32_t Rout, int32_t S) {
  constexpr int U = 16, CH = 256;
  __shared__ double cs[CH * RB];
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int64_t k0 = (int64_t)s * KK / S, k1 = (int64_t)(s + 1) * KK / S;
  double acc[RB];
#pragma unroll
  for (int a = 0; a < RB; ++a) acc[a] = 0.0;
  const TT* col = T + (m < M ? m : 0);
  for (int64_t c0 = k0; c0 < k1; c0 += CH) {
    const int ch = (int)(k1 - c0 < CH ? k1 - c0 : CH);
    __syncthreads();   // the previous chunk has been read
    for (int i = threadIdx.x; i < ch * RB; i += blockDim.x) {
      const int u = i / RB, a = i - u * RB;
      cs[i] = a < Rout ? G[(int64_t)Rout * (c0 + u) + a] : 0.0;
    }
    __syncthreads();
    if (m < M) {
      int u0 = 0;
      for (; u0 + U <= ch; u0 += U) {
        TT x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = col[M * (c0 + u0 + u)];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double xv = to_f64<TT>(x[u]);
          const double* g = cs + (u0 + u) * RB;
#pragma unroll
          for (int a = 0; a < RB; ++a) acc[a] = fma(xv, g[a], acc[a]);
        }
      }
      for (; u0 < ch; ++u0) {
        const double xv = to_f64<TT>(col[M * (c0 + u0)]);
        const double* g = cs + u0 * RB;
#pragma unroll
        for (int a = 0; a < RB; ++a) acc[a] = fma(xv, g[a], acc[a]);
      }
    }
  }
  if (m < M) {
#pragma unroll
    for (int a = 0; a < RB; ++a) {
      if (a >= Rout) break;
      if (S == 1)
        out[m + M * a] = (OT)acc[a];
      else
        part[((int64_t)s * Rout + a) * M + m] = acc[a];
    }
  }
}

// out[e] = sum over the S slices of part[s count + e], FP64, in slice order
template <typename OT>
__global__ void k_sum_slices(const double* __restrict__ part, OT* __restrict__ out, int64_t count, int32_t S) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double acc = 0.0;
  for (int s = 0; s < S; ++s) acc += part[(int64_t)s * count + e];
  out[e] = (OT)acc;
}

// Gram factors of H_k^T H_k in one workgroup: P = G_{<k}^T G_{<k} by the
// recursion P <- sum_j G_i(:, j, :)^T P G_i(:, j, :) over i < k (from
// P = [1]), Q = G_{>k} G_{>k}^T by Q <- sum_j G_i(:, j, :) Q G_i(:, j, :)^T
// over i = d-1 .. k+1 (from Q = [1]).  Out: P at pq (R_k x R_k), Q at
// pq + 256 (R_{k+1} x R_{k+1}), column-major.
__global__ __launch_bounds__(256) void k_tt_grams(CoreDesc cd, int32_t k, double* __restrict__ pq) {
  __shared__ double P[256], U[256], Pn[256];
  const int t = threadIdx.x;
  for (int side = 0; side < 2; ++side) {
    P[t] = t == 0 ? 1.0 : 0.0;
    __syncthreads();
    int rp = 1;   // size of P
    const int lo = side == 0 ? 0 : k + 1, hi = side == 0 ? k : cd.d;
    for (int step = 0; step < hi - lo; ++step) {
      const int i = side == 0 ? lo + step : hi - 1 - step;
      const int r0 = cd.r0[i], ni = cd.n[i], r1 = cd.r1[i];
      const double* Gi = cd.G[i];
      // left: P (r0 x r0) -> (r1 x r1); right: P (r1 x r1) -> (r0 x r0)
      const int rin = side == 0 ? r0 : r1, rout = side == 0 ? r1 : r0;
      Pn[t] = 0.0;
      __syncthreads();
      for (int j = 0; j < ni; ++j) {
        // U(x, y') = sum_x' P(x, x') C(x', y') with C the slice as (rin x rout)
        if (t < rin * rout) {
          const int x = t % rin, yp = t / rin;
          double acc = 0.0;
          for (int xp = 0; xp < rin; ++xp) {
            const double c = side == 0 ? Gi[xp + r0 * (j + (int64_t)ni * yp)] : Gi[yp + r0 * (j + (int64_t)ni * xp)];
            acc += P[x + rin * xp] * c;
          }
          U[x + rin * yp] = acc;
        }
        __syncthreads();
        // Pn(y, y') += sum_x C(x, y) U(x, y')
        if (t < rout * rout) {
          const int y = t % rout, yp = t / rout;
          double acc = 0.0;
          for (int x = 0; x < rin; ++x) {
            const double c = side == 0 ? Gi[x + r0 * (j + (int64_t)ni * y)] : Gi[y + r0 * (j + (int64_t)ni * x)];
            acc += c * U[x + rin * yp];
          }
          Pn[y + rout * yp] += acc;
        }
        __syncthreads();
      }
      P[t] = t < rout * rout ? Pn[t] : 0.0;
      rp = rout;
      __syncthreads();
    }
    (void)rp;
    pq[side * 256 + t] = P[t];
    __syncthreads();
  }
}

// [M | B] for the solve, row-major s x (s + n_k) (row alpha + R_k beta):
// M = Q (x) P (identity when pq is null), B(row, i) = Bc(alpha, i, beta) with
// Bc the right chain's (R_k n_k) x R_{k+1} result.
template <typename WT>
__global__ void k_exact_assemble(const WT* __restrict__ Bc, const double* __restrict__ pq, double* __restrict__ gsum,
                                 int32_t rk, int32_t nk, int32_t rk1) {
  const int s = rk * rk1, ldg = s + nk;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)s * ldg) return;
  const int row = (int)(e / ldg), col = (int)(e - (int64_t)row * ldg);
  const int al = row % rk, be = row / rk;
  double v;
  if (col < s) {
    const int al2 = col % rk, be2 = col / rk;
    v = pq ? pq[256 + be + rk1 * be2] * pq[al + rk * al2] : (row == col ? 1.0 : 0.0);
  } else {
    const int i = col - s;
    v = (double)Bc[al + (int64_t)rk * i + (int64_t)rk * nk * be];
  }
  gsum[e] = v;
}

// A_(k) H_k as n_k x s, column-major: B[i + n_k (alpha + R_k beta)]
template <typename WT>
__global__ void k_exact_rhs_out(const WT* __restrict__ Bc, WT* __restrict__ B, int32_t rk, int32_t nk, int32_t rk1) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nk * rk * rk1;
  if (e >= total) return;
  const int i = (int)(e % nk);
  const int row = (int)(e / nk);
  const int al = row % rk, be = row / rk;
  B[e] = Bc[al + (int64_t)rk * i + (int64_t)rk * nk * be];
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// slices of a contraction: enough workgroups for the device, partials within
// the plan's buffer, at least 64 contracted values per slice
int32_t pick_slices(int64_t groups, int64_t kdim, int64_t count, int64_t part_cap) {
  int64_t S = 1;
  while (groups * S < 2048 && kdim / (2 * S) >= 64 && 2 * S * count <= part_cap) S *= 2;
  return (int32_t)S;
}

template <typename TT, typename WT>
hipError_t fast_t(const tt_plan_s* p, const void* Tv, const double* G, void* outv, int64_t Q, int64_t K, int32_t Rout) {
  const TT* T = static_cast<const TT*>(Tv);
  WT* out = static_cast<WT*>(outv);
  constexpr int NT = 2;
  const int64_t waves = (Q + 16 * NT - 1) / (16 * NT);
  const int64_t blocks = (waves + 3) / 4;
  const int32_t S = pick_slices(blocks, K, Q * Rout, p->ex_part);
  double* part = p->at<double>(p->o_expart);
  const bool vec = K % 4 == 0 && ((uintptr_t)T % (4 * sizeof(TT))) == 0;
  if (vec)
    hipLaunchKernelGGL((k_contract_fast<TT, WT, NT, true>), dim3((unsigned)blocks, (unsigned)S), dim3(256), 0,
                       p->stream, T, G, out, part, Q, K, Rout, S);
  else
    hipLaunchKernelGGL((k_contract_fast<TT, WT, NT, false>), dim3((unsigned)blocks, (unsigned)S), dim3(256), 0,
                       p->stream, T, G, out, part, Q, K, Rout, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 1) return e;
  hipLaunchKernelGGL(k_sum_slices<WT>, dim3(nblk(Q * Rout, 256)), dim3(256), 0, p->stream, part, out, Q * Rout, S);
  return hipGetLastError();
}

template <typename TT, typename WT>
hipError_t slow_t(const tt_plan_s* p, const void* Tv, const double* G, void* outv, int64_t M, int64_t KK,
                  int32_t Rout) {
  const TT* T = static_cast<const TT*>(Tv);
  WT* out = static_cast<WT*>(outv);
  const int64_t blocks = (M + 255) / 256;
  const int32_t S = pick_slices(blocks, KK, M * Rout, p->ex_part);
  double* part = p->at<double>(p->o_expart);
  const dim3 grid((unsigned)blocks, (unsigned)S);
  if (Rout <= 4)
    hipLaunchKernelGGL((k_contract_slow<TT, WT, 4>), grid, dim3(256), 0, p->stream, T, G, out, part, M, KK, Rout, S);
  else if (Rout <= 8)
    hipLaunchKernelGGL((k_contract_slow<TT, WT, 8>), grid, dim3(256), 0, p->stream, T, G, out, part, M, KK, Rout, S);
  else if (Rout <= 12)
    hipLaunchKernelGGL((k_contract_slow<TT, WT, 12>), grid, dim3(256), 0, p->stream, T, G, out, part, M, KK, Rout, S);
  else
    hipLaunchKernelGGL((k_contract_slow<TT, WT, 16>), grid, dim3(256), 0, p->stream, T, G, out, part, M, KK, Rout, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 1) return e;
  hipLaunchKernelGGL(k_sum_slices<WT>, dim3(nblk(M * Rout, 256)), dim3(256), 0, p->stream, part, out, M * Rout, S);
  return hipGetLastError();
}

// one contraction step on input of storage type xdt (X itself) or the work type
template <typename TT, typename WT>
hipError_t merged_t(const tt_plan_s* p, const void* Tv, const double* G, void* outv, int64_t M, int64_t KK,
                    int32_t Rout) {
  const TT* T = static_cast<const TT*>(Tv);
  WT* out = static_cast<WT*>(outv);
  const int64_t blocks = (M + 255) / 256;
  const int32_t S = pick_slices(blocks, KK, M * Rout, p->ex_part);
  double* part = p->at<double>(p->o_expart);
  const dim3 grid((unsigned)blocks, (unsigned)S);
  if (Rout <= 4)
    hipLaunchKernelGGL((k_contract_merged<TT, WT, 4>), grid, dim3(256), 0, p->stream, T, G, out, part, M, KK, Rout, S);
  else if (Rout <= 8)
    hipLaunchKernelGGL((k_contract_merged<TT, WT, 8>), grid, dim3(256), 0, p->stream, T, G, out, part, M, KK, Rout, S);
  else if (Rout <= 12)
    hipLaunchKernelGGL((k_contract_merged<TT, WT, 12>), grid, dim3(256), 0, p->stream, T, G, out, part, M, KK, Rout,
                       S);
  else
    hipLaunchKernelGGL((k_contract_merged<TT, WT, 16>), grid, dim3(256), 0, p->stream, T, G, out, part, M, KK, Rout,
                       S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 1) return e;
  hipLaunchKernelGGL(k_sum_slices<WT>, dim3(nblk(M * Rout, 256)), dim3(256), 0, p->stream, part, out, M * Rout, S);
  return hipGetLastError();
}

hipError_t contract_merged(const tt_plan_s* p, bool input_is_x, const void* T, const double* C, void* out, int64_t M,
                           int64_t KK, int32_t Rout) {
  const tt_dtype it = input_is_x ? p->xdt : p->wdt;
  if (p->wdt == TT_F64) {
    if (it == TT_F64) return merged_t<double, double>(p, T, C, out, M, KK, Rout);
    if (it == TT_F32) return merged_t<float, double>(p, T, C, out, M, KK, Rout);
    return merged_t<uint16_t, double>(p, T, C, out, M, KK, Rout);
  }
  if (it == TT_F64) return merged_t<double, float>(p, T, C, out, M, KK, Rout);
  if (it == TT_F32) return merged_t<float, float>(p, T, C, out, M, KK, Rout);
  return merged_t<uint16_t, float>(p, T, C, out, M, KK, Rout);
}

hipError_t contract(const tt_plan_s* p, bool fast, bool input_is_x, const void* T, const double* G, void* out,
                    int64_t a, int64_t b, int32_t Rout) {
  const tt_dtype it = input_is_x ? p->xdt : p->wdt;
  if (p->wdt == TT_F64) {
    if (it == TT_F64) return fast ? fast_t<double, double>(p, T, G, out, a, b, Rout) : slow_t<double, double>(p, T, G, out, a, b, Rout);
    if (it == TT_F32) return fast ? fast_t<float, double>(p, T, G, out, a, b, Rout) : slow_t<float, double>(p, T, G, out, a, b, Rout);
    return fast ? fast_t<uint16_t, double>(p, T, G, out, a, b, Rout) : slow_t<uint16_t, double>(p, T, G, out, a, b, Rout);
  }
  if (it == TT_F64) return fast ? fast_t<double, float>(p, T, G, out, a, b, Rout) : slow_t<double, float>(p, T, G, out, a, b, Rout);
  if (it == TT_F32) return fast ? fast_t<float, float>(p, T, G, out, a, b, Rout) : slow_t<float, float>(p, T, G, out, a, b, Rout);
  return fast ? fast_t<uint16_t, float>(p, T, G, out, a, b, Rout) : slow_t<uint16_t, float>(p, T, G, out, a, b, Rout);
}

// C(a, i + n_a j) = sum_b Ga(a, i, b) Gb(b, j, 0): the last two cores merged
// into one core of shape (R_a, n_a n_b, 1), so that the first step of a right
// chain contracts both slow modes in one pass over its input and writes
// R_a N' / (n_a n_b) values instead of R_b N' / n_b (N' the input's size):
// on an X-sized input the large intermediate write, which costs HBM time in
// a read stream, disappears.  FP64, one thread per entry.
__global__ void k_merge_cores(const double* __restrict__ Ga, const double* __restrict__ Gb, double* __restrict__ C,
                              int32_t Ra, int32_t na, int32_t Rb, int32_t nb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)Ra * na * nb;
  if (e >= total) return;
  const int32_t a = (int32_t)(e % Ra);
  const int64_t ij = e / Ra;
  const int32_t i = (int32_t)(ij % na), j = (int32_t)(ij / na);
  double s = 0.0;
  for (int b = 0; b < Rb; ++b) s = fma(Ga[a + (int64_t)Ra * (i + (int64_t)na * b)], Gb[b + (int64_t)Rb * j], s);
  C[e] = s;
}

}  // namespace

// Doubles of the merged last two cores (0 when the plan has fewer than 3
// modes or the merged core would exceed 2^23 doubles)
int64_t tt_exact_merge_doubles(const tt_plan_s* p) {
  const int d = p->d;
  if (d < 3) return 0;
  const int64_t c = p->r[d - 2] * p->n[d - 2] * p->n[d - 1];
  return c <= ((int64_t)1 << 23) ? c : 0;
}

// Sizes of the exact path's buffers (work-type values): the left interfaces
// Phi_1 .. Phi_{d-1} and the right chains of every Phi_k.
void tt_exact_sizes(const tt_plan_s* p, int64_t* phi, int64_t* chain) {
  const int d = p->d;
  int64_t ph = 1, ch = 1;
  for (int k = 0; k < d; ++k) {
    int64_t tail = 1;   // prod_{i >= k} n_i
    for (int i = k; i < d; ++i) tail *= p->n[i];
    if (k >= 1 && p->r[k] * tail > ph) ph = p->r[k] * tail;
    // right chain on Phi_k: after contracting modes d-1 .. s, M = R_k prod_{k <= i < s} n_i, R_s ranks
    int64_t M = p->r[k] * tail;
    for (int s = d - 1; s > k; --s) {
      M /= p->n[s];
      if (M * p->r[s] > ch) ch = M * p->r[s];
    }
  }
  *phi = ph;
  *chain = ch;
}

// Phi_{k+1} = Phi_k contracted over (alpha, i_k) with core k.
hipError_t launch_exact_left(const tt_plan_s* p, const void* phi_k, bool is_x, int k, const double* Gk, void* phi_next) {
  int64_t Q = 1;
  for (int i = k + 1; i < p->d; ++i) Q *= p->n[i];
  return contract(p, true, is_x, phi_k, Gk, phi_next, Q, p->r[k] * p->n[k], (int32_t)p->r[k + 1]);
}

// B_k (R_k n_k x R_{k+1}) = Phi_k contracted over modes d-1 .. k+1 with their
// cores; the chain alternates between the two chain buffers.  Returns the
// buffer holding B_k in *result (Phi_k itself when k = d - 1).
hipError_t launch_exact_right(const tt_plan_s* p, const void* phi_k, bool is_x, int k, const double* const* G,
                              const void** result) {
  const int d = p->d;
  int64_t M = p->r[k];
  for (int i = k; i < d; ++i) M *= p->n[i];
  const void* cur = phi_k;
  bool cur_x = is_x;
  char* bufs[2] = {p->ws + p->o_exch, p->ws + p->o_exch + p->wsize() * p->ex_chain};
  int which = 0;
  int s = d - 1;
  if (p->o_exmerge && d - 2 > k) {
    // modes d-1 and d-2 in one pass, through the merged core (R_d = 1)
    double* C = p->at<double>(p->o_exmerge);
    const int32_t Ra = (int32_t)p->r[d - 2], na = (int32_t)p->n[d - 2], Rb = (int32_t)p->r[d - 1],
                  nb = (int32_t)p->n[d - 1];
    hipLaunchKernelGGL(k_merge_cores, dim3(nblk((int64_t)Ra * na * nb, 256)), dim3(256), 0, p->stream, G[d - 2],
                       G[d - 1], C, Ra, na, Rb, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    M /= (int64_t)na * nb;
    if ((e = contract_merged(p, cur_x, cur, C, bufs[which], M, (int64_t)na * nb, Ra)) != hipSuccess) return e;
    cur = bufs[which];
    cur_x = false;
    which ^= 1;
    s = d - 3;
  }
  for (; s > k; --s) {
    M /= p->n[s];
    const int64_t KK = p->n[s] * p->r[s + 1];
    hipError_t e = contract(p, false, cur_x, cur, G[s], bufs[which], M, KK, (int32_t)p->r[s]);
    if (e != hipSuccess) return e;
    cur = bufs[which];
    cur_x = false;
    which ^= 1;
  }
  if (cur_x) return hipErrorInvalidValue;   // k = d - 1 with Phi_k = X (d = 1): not a valid plan
  *result = cur;
  return hipSuccess;
}

hipError_t launch_exact_grams(const tt_plan_s* p, const CoreDesc& cd, int k) {
  hipLaunchKernelGGL(k_tt_grams, dim3(1), dim3(256), 0, p->stream, cd, (int32_t)k, p->at<double>(p->o_exgram));
  return hipGetLastError();
}

hipError_t launch_exact_assemble(const tt_plan_s* p, int k, const void* Bc, bool use_grams) {
  const int32_t rk = (int32_t)p->r[k], nk = (int32_t)p->n[k], rk1 = (int32_t)p->r[k + 1];
  const int64_t count = (int64_t)rk * rk1 * (rk * rk1 + nk);
  const double* pq = use_grams ? p->at<double>(p->o_exgram) : nullptr;
  if (p->wdt == TT_F64)
    hipLaunchKernelGGL(k_exact_assemble<double>, dim3(nblk(count, 256)), dim3(256), 0, p->stream,
                       static_cast<const double*>(Bc), pq, p->at<double>(p->o_gsum), rk, nk, rk1);
  else
    hipLaunchKernelGGL(k_exact_assemble<float>, dim3(nblk(count, 256)), dim3(256), 0, p->stream,
                       static_cast<const float*>(Bc), pq, p->at<double>(p->o_gsum), rk, nk, rk1);
  return hipGetLastError();
}

hipError_t launch_exact_rhs_out(const tt_plan_s* p, int k, const void* Bc, void* B) {
  const int32_t rk = (int32_t)p->r[k], nk = (int32_t)p->n[k], rk1 = (int32_t)p->r[k + 1];
  const int64_t count = (int64_t)nk * rk * rk1;
  if (p->wdt == TT_F64)
    hipLaunchKernelGGL(k_exact_rhs_out<double>, dim3(nblk(count, 256)), dim3(256), 0, p->stream,
                       static_cast<const double*>(Bc), static_cast<double*>(B), rk, nk, rk1);
  else
    hipLaunchKernelGGL(k_exact_rhs_out<float>, dim3(nblk(count, 256)), dim3(256), 0, p->stream,
                       static_cast<const float*>(Bc), static_cast<float*>(B), rk, nk, rk1);
  return hipGetLastError();
}
