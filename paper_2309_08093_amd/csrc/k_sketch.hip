// Data sketch Y_k = S_{-k} A_(k)^T (Sec. 3, eq. (3.4); TensorSketch of
// Sec. 2.2): a sign-weighted scatter-add of every entry of X into J buckets.
//
// X is read as a sequence of mode-0 fibres (n_0 contiguous entries).  Within a
// fibre only i_0 varies, so the hash contribution of every other mode is one
// wave-uniform packed key per fibre; lane l owns positions i_0 = l + 64 j and
// keeps their packed table entries in registers.
//
//  * k >= 1: one workgroup owns one column i_k of Y and a chunk of that
//    column's fibres; it accumulates into a J-entry LDS array with LDS
//    atomics and writes the array to a partial buffer.  A second kernel sums
//    the partials of each column in FP64 in a fixed order.
//  * k = 0: a fibre has one bucket (its entries differ only in i_0, the
//    unsketched mode), so one workgroup owns one bucket b and gathers the
//    fibres hashed to b: for each i_1 it visits the outer tuples (modes 2..d-1)
//    whose partial hash is (b - h_1(i_1)) mod J, found in a bucket-sorted list.
//    Accumulation is in registers; no atomics.
#include "tt_internal.h"

namespace {

__device__ __forceinline__ uint32_t key_add(uint32_t a, uint32_t b, uint32_t J) {
  uint32_t s = (a & TT_KEY_MASK) + (b & TT_KEY_MASK);
  s = s >= J ? s - J : s;
  return s | ((a ^ b) & TT_KEY_SIGN);
}

template <typename WT>
__device__ __forceinline__ WT to_work(double v) { return (WT)v; }
template <typename WT>
__device__ __forceinline__ WT to_work(float v) { return (WT)v; }
template <typename WT>
__device__ __forceinline__ WT to_work(uint16_t v) { return (WT)__uint_as_float((uint32_t)v << 16); }

template <typename WT>
__device__ __forceinline__ WT apply_sign(WT x, uint32_t key) { return (key & TT_KEY_SIGN) ? -x : x; }

// ---------------------------------------------------------------- k >= 1
template <typename XT, typename WT, int NJ, int U>
__global__ __launch_bounds__(256) void k_sketch_modek(
    const XT* __restrict__ X, const uint32_t* __restrict__ tab0, const uint32_t* __restrict__ KI,
    const uint32_t* __restrict__ KO, WT* __restrict__ part, int32_t n0, int32_t nk, int64_t M, int64_t F,
    uint32_t J, int32_t S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  WT* acc = reinterpret_cast<WT*>(smem_raw);
  const int col = blockIdx.x;
  const int chunk = blockIdx.y;
  for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) acc[b] = (WT)0;

  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int W = blockDim.x >> 6;
  uint32_t t0[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int i0 = lane + 64 * j;
    t0[j] = i0 < n0 ? tab0[i0] : 0u;
  }
  const int64_t q0 = F * chunk / S, q1 = F * (chunk + 1) / S;
  const int64_t qa = q0 + (q1 - q0) * w / W, qe = q0 + (q1 - q0) * (w + 1) / W;
  __syncthreads();

  int64_t mu = qa % M, rho = qa / M;
  for (int64_t q = qa; q < qe; q += U) {
    const XT* base[U];
    uint32_t kf[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = q + u < qe;
      kf[u] = ok[u] ? key_add(KI[mu], KO[rho], J) : 0u;
      base[u] = X + (((rho * nk + col) * M + mu) * (int64_t)n0);
      if (++mu == M) { mu = 0; ++rho; }
    }
    XT v[U][NJ];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int i0 = lane + 64 * j;
        v[u][j] = (ok[u] && i0 < n0) ? base[u][i0] : (XT)0;
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int i0 = lane + 64 * j;
        if (ok[u] && i0 < n0) {
          const uint32_t key = key_add(t0[j], kf[u], J);
          atomicAdd(&acc[key & TT_KEY_MASK], apply_sign<WT>(to_work<WT>(v[u][j]), key));
        }
      }
  }
  __syncthreads();
  WT* out = part + ((int64_t)col * S + chunk) * (int64_t)J;
  for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) out[b] = acc[b];
}

// Y[b + J i] = sum_c part[(i S + c) J + b], summed in FP64 in chunk order.
template <typename WT>
__global__ void k_reduce_parts(const WT* __restrict__ part, WT* __restrict__ Y, int64_t J, int64_t nk, int32_t S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= J * nk) return;
  const int64_t i = idx / J, b = idx - i * J;
  const WT* p = part + i * S * J + b;
  double s = 0.0;
  for (int c = 0; c < S; ++c) s += (double)p[(int64_t)c * J];
  Y[idx] = (WT)s;
}

// ---------------------------------------------------------------- k = 0
template <typename XT, typename WT, int NJ, int U>
__global__ __launch_bounds__(256) void k_sketch_mode0(
    const XT* __restrict__ X, const uint32_t* __restrict__ tab1, const uint32_t* __restrict__ off,
    const uint32_t* __restrict__ sorted, WT* __restrict__ Y, int32_t n0, int32_t n1, uint32_t J,
    int32_t i0_lo, int32_t i0_cnt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  WT* red = reinterpret_cast<WT*>(smem_raw);   // W x (NJ*64)
  const uint32_t b = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int W = blockDim.x >> 6;
  WT acc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) acc[j] = (WT)0;

  for (int i1 = w; i1 < n1; i1 += W) {
    const uint32_t t1 = tab1[i1];
    const uint32_t h1 = t1 & TT_KEY_MASK;
    const uint32_t c = b >= h1 ? b - h1 : b + J - h1;
    const uint32_t beg = off[c], end = off[c + 1];
    for (uint32_t e = beg; e < end; e += U) {
      uint32_t item[U];
      XT v[U][NJ];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = e + u < end;
        item[u] = ok ? sorted[e + u] : 0u;
        const XT* base = X + ((int64_t)(item[u] & TT_KEY_MASK) * n1 + i1) * (int64_t)n0 + i0_lo;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int i0 = lane + 64 * j;
          v[u][j] = (ok && i0 < i0_cnt) ? base[i0] : (XT)0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[j] += apply_sign<WT>(to_work<WT>(v[u][j]), item[u] ^ t1);
    }
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) red[w * (NJ * 64) + j * 64 + lane] = acc[j];
  __syncthreads();
  for (int i = threadIdx.x; i < i0_cnt; i += blockDim.x) {
    WT s = (WT)0;
    for (int ww = 0; ww < W; ++ww) s += red[ww * (NJ * 64) + i];
    Y[(int64_t)b + (int64_t)J * (i0_lo + i)] = s;
  }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename XT, typename WT, int NJ>
hipError_t run_modek(const tt_plan_s* p, const XT* X, int k, WT* Y) {
  constexpr int U = NJ >= 8 ? 1 : 8 / NJ;
  const int64_t n0 = p->n[0], nk = p->n[k];
  int64_t M = 1, Rk = 1;
  for (int s = 1; s < k; ++s) M *= p->n[s];
  for (int s = k + 1; s < p->d; ++s) Rk *= p->n[s];
  const int64_t F = M * Rk;
  const int64_t S = tt_sketch_chunks(p, k);
  uint32_t* KI = p->at<uint32_t>(p->o_KI);
  uint32_t* KO = p->at<uint32_t>(p->o_KO);
  hipError_t e;
  // an empty mode range yields the single key 0 (bucket 0, sign +)
  if ((e = launch_build_keys(p, KI, M, 1, k - 1)) != hipSuccess) return e;
  if ((e = launch_build_keys(p, KO, Rk, k + 1, p->d - 1)) != hipSuccess) return e;
  WT* part = p->at<WT>(p->o_part);
  const uint32_t* tab0 = p->at<uint32_t>(p->o_tab) + p->tab_off[0];
  const size_t lds = (size_t)p->J * sizeof(WT);
  hipLaunchKernelGGL((k_sketch_modek<XT, WT, NJ, U>), dim3((unsigned)nk, (unsigned)S), dim3(256), lds, p->stream,
                     X, tab0, KI, KO, part, (int32_t)n0, (int32_t)nk, M, F, (uint32_t)p->J, (int32_t)S);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((k_reduce_parts<WT>), dim3(nblk(p->J * nk, 256)), dim3(256), 0, p->stream, part, Y, p->J, nk,
                     (int32_t)S);
  return hipGetLastError();
}

template <typename XT, typename WT, int NJ>
hipError_t run_mode0(const tt_plan_s* p, const XT* X, WT* Y) {
  constexpr int U = NJ >= 8 ? 1 : 8 / NJ;
  hipError_t e = launch_outer_sort(p);
  if (e != hipSuccess) return e;
  const int64_t n0 = p->n[0], n1 = p->n[1];
  const uint32_t* tab1 = p->at<uint32_t>(p->o_tab) + p->tab_off[1];
  const uint32_t* off = p->at<uint32_t>(p->o_cnt);
  const uint32_t* sorted = p->at<uint32_t>(p->o_sortO);
  constexpr int CH = NJ * 64;
  const size_t lds = (size_t)4 * CH * sizeof(WT);
  for (int64_t lo = 0; lo < n0; lo += CH) {
    const int64_t cnt = (n0 - lo) < CH ? (n0 - lo) : CH;
    hipLaunchKernelGGL((k_sketch_mode0<XT, WT, NJ, U>), dim3((unsigned)p->J), dim3(256), lds, p->stream, X, tab1, off,
                       sorted, Y, (int32_t)n0, (int32_t)n1, (uint32_t)p->J, (int32_t)lo, (int32_t)cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename XT, typename WT>
hipError_t dispatch(const tt_plan_s* p, const void* Xv, int k, void* Yv) {
  const XT* X = static_cast<const XT*>(Xv);
  WT* Y = static_cast<WT*>(Yv);
  const int64_t n0 = p->n[0];
  if (k == 0) {
    // chunks of at most 1024 positions of i_0 per launch
    if (n0 <= 64) return run_mode0<XT, WT, 1>(p, X, Y);
    if (n0 <= 128) return run_mode0<XT, WT, 2>(p, X, Y);
    if (n0 <= 256) return run_mode0<XT, WT, 4>(p, X, Y);
    if (n0 <= 512) return run_mode0<XT, WT, 8>(p, X, Y);
    return run_mode0<XT, WT, 16>(p, X, Y);
  }
  if (n0 <= 64) return run_modek<XT, WT, 1>(p, X, k, Y);
  if (n0 <= 128) return run_modek<XT, WT, 2>(p, X, k, Y);
  if (n0 <= 256) return run_modek<XT, WT, 4>(p, X, k, Y);
  if (n0 <= 512) return run_modek<XT, WT, 8>(p, X, k, Y);
  if (n0 <= 1024) return run_modek<XT, WT, 16>(p, X, k, Y);
  if (n0 <= 2048) return run_modek<XT, WT, 32>(p, X, k, Y);
  return run_modek<XT, WT, 64>(p, X, k, Y);
}

}  // namespace

// Number of fibre chunks per column for k >= 1 (also sizes the partials).
int64_t tt_sketch_chunks(const tt_plan_s* p, int k) {
  int64_t M = 1, Rk = 1;
  for (int s = 1; s < k; ++s) M *= p->n[s];
  for (int s = k + 1; s < p->d; ++s) Rk *= p->n[s];
  const int64_t F = M * Rk;
  int64_t S = (2048 + p->n[k] - 1) / p->n[k];
  if (S > F) S = F;
  return S < 1 ? 1 : S;
}

hipError_t launch_sketch_tensor(const tt_plan_s* p, const void* X, int k, void* Y) {
  if (p->wdt == TT_F64) {
    if (p->xdt == TT_F64) return dispatch<double, double>(p, X, k, Y);
    if (p->xdt == TT_F32) return dispatch<float, double>(p, X, k, Y);
    return dispatch<uint16_t, double>(p, X, k, Y);
  }
  if (p->xdt == TT_F64) return dispatch<double, float>(p, X, k, Y);
  if (p->xdt == TT_F32) return dispatch<float, float>(p, X, k, Y);
  return dispatch<uint16_t, float>(p, X, k, Y);
}
