// Batched form: many independent TT-TS problems of uneven shapes and ranks
// advance together, one sweep step at a time.
//
// Each problem keeps its own plan (tables, cores, interface and solve
// buffers) in a slice of one batch workspace.  Per step k of a sweep:
//  * the interface sketches (and the new transform of core k - 1) of all
//    problems with order > k are one launch per kernel (core FFTs, chain
//    products, face-splitting inverse FFTs), one workgroup per (problem,
//    column), each problem with its own J and FFT plan from a per-step
//    descriptor;
//  * the core updates of all those problems are one launch per kernel: the
//    Gram contraction, the summed partials, the Cholesky factorisation, the
//    substitution, QR (one launch per register shape; blocks too tall for
//    registers per problem) and the absorb of R, each with one workgroup (or
//    block set) per problem, driven by per-step descriptors in device memory;
//  * the data sketches of all those problems are ONE persistent launch:
//    - k >= 1: the units (mode-0 fibres; for k >= 2 the contiguous
//      n_0 x n_1 slabs) of every participating problem, problem by problem
//      and column by column, form one sequence that is split into equal
//      contiguous ranges, one per workgroup.  A workgroup accumulates the part
//      of a column it holds in a J-entry FP64 LDS array (keys computed on the
//      fly from the tables) and writes it as one partial of that column; a
//      second launch adds the partials of each column in a fixed order;
//    - k = 0: one workgroup per (problem, bucket) gathers the fibres hashed to
//      the bucket from the problem's bucket-sorted list of outer tuples.  For
//      the problems whose plans take Y_1 from the outer sketch (J n_0 n_1
//      small beside X) a workgroup per (problem, bucket) instead sums the
//      whole n_0 x n_1 slabs of its outer tuples into that sketch, and Y_0
//      and Y_1 are both formed from it, so X is read once for the two steps.
// The data sketches of every step need only X and the sweep's tables, so they
// all run first, on a side stream, and step k's core updates wait for step
// k's sketch.  A whole sweep can be captured once into a hipGraph and
// replayed; the table
// generator then reads the sweep index from a device counter that the graph
// advances.  The workgroup count of each k >= 1 launch is chosen by
// tt_batch_autotune from timed candidates.
#include <algorithm>
#include <type_traits>
#include <new>
#include <vector>

#include "tt_internal.h"

namespace {

struct BTensor {
  const float* X;
  float* Y;                  // the plan's all-mode Y buffer: Y_k (J x n_k, column-major) at J * toff[k]
  const uint32_t* tab;       // packed tables of all modes
  const uint32_t* off;       // k = 0: bucket offsets of the outer tuples (J + 1)
  const uint32_t* sorted;    // k = 0: outer tuples sorted by bucket
  float* zo;                 // problems whose Y_1 comes from the k = 0 pass: its outer sketch, else null
  const uint2* sl[TT_MAX_ORDER];   // k >= 2: the slabs of a mode-k column sorted by key
  int32_t n[TT_MAX_ORDER];
  int32_t toff[TT_MAX_ORDER];
  int32_t d;
  uint32_t J;
};

__device__ __forceinline__ uint32_t key_add(uint32_t a, uint32_t b, uint32_t J) {
  uint32_t s = (a & TT_KEY_MASK) + (b & TT_KEY_MASK);
  s = s >= J ? s - J : s;
  return s | ((a ^ b) & TT_KEY_SIGN);
}

__device__ __forceinline__ double signed_f64(float x, uint32_t s) {
  return (double)__uint_as_float(__float_as_uint(x) ^ s);
}

__device__ __forceinline__ int64_t owner(int64_t g, int64_t W, int64_t Ftot) { return ((g + 1) * W - 1) / Ftot; }

// Descriptor pointers are plain (generic) pointers; reading X through the
// global address space keeps its loads off the LDS wait counter, so the
// shuffles and LDS atomics between them do not wait for the loads.
typedef const float __attribute__((address_space(1)))* gfloat;
typedef const uint32_t __attribute__((address_space(1)))* guint;

// index of the segment of a non-decreasing prefix array (n + 1 entries) that holds g
__device__ __forceinline__ int seg_of(const int64_t* pre, int n, int64_t g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// lanes per fibre (log2): the smallest power of two whose NJ entries per lane
// cover the fibre, at most 64
template <int NJ>
__device__ __forceinline__ int lpf_log2_of(int n0) {
  int l = 0;
  while ((NJ << l) < n0 && l < 6) ++l;
  return l;
}

// V-wide loads of FP32 values (V = 1, 2, 4)
template <int V> struct FVec;
template <> struct FVec<1> { typedef float T; };
template <> struct FVec<2> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct FVec<4> { typedef float T __attribute__((ext_vector_type(4))); };
template <int V> __device__ __forceinline__ float lane_of(const typename FVec<V>::T& a, int i) { return a[i]; }
template <> __device__ __forceinline__ float lane_of<1>(const float& a, int) { return a; }

// ---------------------------------------------------------------- k >= 1
// NJ: entries of a fibre per lane; FIB: fibres per lane group per load batch
// (both chosen per step by the autotuner)
template <int NJ, int FIB>
__global__ __launch_bounds__(256) void k_bsketch_k(const BTensor* __restrict__ T, const int32_t* __restrict__ tids,
                                                   const int64_t* __restrict__ fpre, const int64_t* __restrict__ cpre,
                                                   const int64_t* __restrict__ spre, int32_t nt, int32_t k,
                                                   double* __restrict__ part, int32_t Jmax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  const int64_t W = gridDim.x, w = blockIdx.x;
  const int64_t Ttot = fpre[nt];
  const int64_t gs = w * Ttot / W, ge = (w + 1) * Ttot / W;
  if (gs >= ge) return;
  int j = seg_of(fpre, nt, gs);
  int64_t g = gs;
  while (g < ge) {
    while (fpre[j + 1] <= g) ++j;
    const BTensor& t = T[tids[j]];
    const int d = t.d, n0 = t.n[0], nk = t.n[k];
    const uint32_t J = t.J;
    int64_t M = 1, R = 1;
    for (int s = 1; s < k; ++s) M *= t.n[s];
    for (int s = k + 1; s < d; ++s) R *= t.n[s];
    const int64_t F = M * R;
    const int lpf_log2 = lpf_log2_of<NJ>(n0);
    const int LPF = 1 << lpf_log2, G = 64 >> lpf_log2;
    const int gi = lane >> lpf_log2, v = lane & (LPF - 1);
    const gfloat Xg = (gfloat)t.X;
    const guint tabg = (guint)t.tab;
    uint32_t tb[NJ], ts[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
      const int i0 = v + LPF * q;
      const uint32_t e = i0 < n0 ? tabg[t.toff[0] + i0] : 0u;
      tb[q] = e & TT_KEY_MASK;
      ts[q] = e & TT_KEY_SIGN;
    }
    const int64_t q0 = g - fpre[j];
    const int64_t c = q0 / F;
    const int64_t qa = q0 - c * F;
    const int64_t lim = ge - fpre[j] - c * F;
    const int64_t qe = lim < F ? lim : F;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) acc[b] = 0.0;
    __syncthreads();
    const int64_t wa = qa + (qe - qa) * wv / NW, we = qa + (qe - qa) * (wv + 1) / NW;
    for (int64_t fb = wa; fb < we; fb += 64) {
      // key and element offset of the next (up to) 64 fibres, one per lane
      const int64_t fl = fb + lane;
      uint32_t keyl = 0;
      int64_t offl = 0;
      if (fl < we) {
        // a problem's fibre indices fit in 32 bits (its size is checked at plan time)
        const uint32_t M32 = (uint32_t)M;
        uint32_t rho = (uint32_t)fl / M32, mu = (uint32_t)fl - rho * M32;
        offl = (((int64_t)rho * nk + c) * M + mu) * (int64_t)n0;
        for (int s = 1; s < k; ++s) {
          const uint32_t ns = (uint32_t)t.n[s];
          const uint32_t q = mu / ns;
          keyl = key_add(keyl, tabg[t.toff[s] + (mu - q * ns)], J);
          mu = q;
        }
        for (int s = k + 1; s < d; ++s) {
          const uint32_t ns = (uint32_t)t.n[s];
          const uint32_t q = rho / ns;
          keyl = key_add(keyl, tabg[t.toff[s] + (rho - q * ns)], J);
          rho = q;
        }
      }
      const int nb = (we - fb) < 64 ? (int)(we - fb) : 64;
      // FIB fibres per lane group in flight: short fibres need many loads
      // outstanding per wave to cover the memory latency
      for (int u0 = 0; u0 < nb; u0 += FIB * G) {
        float x[FIB][NJ];
        uint32_t kb[FIB], ks[FIB];
        bool ok[FIB];
#pragma unroll
        for (int u = 0; u < FIB; ++u) {
          const int idx = u0 + u * G + gi;
          ok[u] = idx < nb;
          const uint32_t key = (uint32_t)__shfl((int)keyl, idx & 63, 64);
          kb[u] = key & TT_KEY_MASK;
          ks[u] = key & TT_KEY_SIGN;
          const int lo = __shfl((int)(uint32_t)(uint64_t)offl, idx & 63, 64);
          const int hi = __shfl((int)(uint32_t)((uint64_t)offl >> 32), idx & 63, 64);
          const int64_t off = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
#pragma unroll
          for (int q = 0; q < NJ; ++q) {   // lanes past the fibre stay masked off (no load issued)
            const int i0 = v + LPF * q;
            x[u][q] = (ok[u] && i0 < n0) ? __builtin_nontemporal_load(Xg + off + i0) : 0.0f;
          }
        }
#pragma unroll
        for (int u = 0; u < FIB; ++u)
#pragma unroll
          for (int q = 0; q < NJ; ++q) {
            const int i0 = v + LPF * q;
            if (ok[u] && i0 < n0) {
              uint32_t bk = tb[q] + kb[u];
              bk = bk >= J ? bk - J : bk;
              atomicAdd(&acc[bk], signed_f64(x[u][q], ts[q] ^ ks[u]));
            }
          }
      }
    }
    __syncthreads();
    const int64_t gc = cpre[j] + c;
    const int64_t slot = w - owner(fpre[j] + c * F, W, Ttot);
    double* out = part + (spre[gc] + slot) * (int64_t)Jmax;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) out[b] = acc[b];
    __syncthreads();
    g = fpre[j] + c * F + qe;
  }
}

// ---------------------------------------------------------------- k >= 2, slabs
// For k >= 2 the n_0 x n_1 entries with fixed (i_2, ..., i_{d-1}) (a slab) are
// contiguous in X, and entry e = i_0 + n_0 i_1 of a slab lands in bucket
// P[e] + K, with P[e] = h_0(i_0) + h_1(i_1) (a per-problem LDS table) and K
// the sum of the tables of the other modes but k (one value per slab).  The
// unit of work is the slab instead of the fibre: the lanes of a wave stream
// through the entries of its slab range 64 at a time, so every load is a full
// coalesced row and no per-fibre key or offset is exchanged between lanes.
// A lane recomputes K (from the mode tables, copied to LDS) only when it
// steps into another slab.
constexpr size_t kSlabLds = 48 << 10;   // bytes for the slab table and the mode tables

// U: 64-entry rows per lane in flight (chosen per step by the autotuner)
template <int U>
__global__ __launch_bounds__(256) void k_bsketch_slab(const BTensor* __restrict__ T, const int32_t* __restrict__ tids,
                                                      const int64_t* __restrict__ fpre, const int64_t* __restrict__ cpre,
                                                      const int64_t* __restrict__ spre, int32_t nt, int32_t k,
                                                      double* __restrict__ part, int32_t Jmax, int32_t Smax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  uint32_t* P = reinterpret_cast<uint32_t*>(acc + Jmax);   // Smax entries
  uint32_t* tl = P + Smax;                                  // the problem's packed tables
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  const int64_t W = gridDim.x, w = blockIdx.x;
  const int64_t Ttot = fpre[nt];
  const int64_t gs = w * Ttot / W, ge = (w + 1) * Ttot / W;
  if (gs >= ge) return;
  int j = seg_of(fpre, nt, gs), jp = -1;
  int64_t g = gs;
  while (g < ge) {
    while (fpre[j + 1] <= g) ++j;
    const BTensor& t = T[tids[j]];
    const int d = t.d;
    const uint32_t n0 = (uint32_t)t.n[0], n1 = (uint32_t)t.n[1], nk = (uint32_t)t.n[k];
    const uint32_t S = n0 * n1;
    const uint32_t J = t.J;
    int64_t Mp = 1, R = 1;
    for (int s = 2; s < k; ++s) Mp *= t.n[s];
    for (int s = k + 1; s < d; ++s) R *= t.n[s];
    const int64_t F = Mp * R;   // slabs per column
    const int64_t q0 = g - fpre[j];
    const int64_t c = q0 / F;
    const int64_t qa = q0 - c * F;
    const int64_t lim = ge - fpre[j] - c * F;
    const int64_t qe = lim < F ? lim : F;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) acc[b] = 0.0;
    if (j != jp) {   // P and the tables of a new problem (no wave reads them here)
      const int ntab = t.toff[d - 1] + t.n[d - 1];
      for (int i = threadIdx.x; i < ntab; i += blockDim.x) tl[i] = t.tab[i];
      __syncthreads();
      for (uint32_t e = threadIdx.x; e < S; e += blockDim.x) {
        const uint32_t i1 = e / n0;
        P[e] = key_add(tl[t.toff[0] + (e - i1 * n0)], tl[t.toff[1] + i1], J);
      }
      jp = j;
    }
    __syncthreads();
    const int64_t wa = qa + (qe - qa) * wv / NW, we = qa + (qe - qa) * (wv + 1) / NW;
    const int64_t tot = (we - wa) * (int64_t)S;
    const gfloat Xg = (gfloat)t.X;
    const uint32_t Mp32 = (uint32_t)Mp;
    // offset and key of slab sl of column c (sl < F; slab indices of a
    // problem fit in 32 bits)
    auto locate = [&](int64_t sl, int64_t& base, uint32_t& K) {
      uint32_t rho = (uint32_t)sl / Mp32, mu = (uint32_t)sl - rho * Mp32;
      base = (((int64_t)rho * nk + c) * Mp + mu) * (int64_t)S;
      K = 0;
      for (int s = 2; s < k; ++s) {
        const uint32_t ns = (uint32_t)t.n[s], q = mu / ns;
        K = key_add(K, tl[t.toff[s] + (mu - q * ns)], J);
        mu = q;
      }
      for (int s = k + 1; s < d; ++s) {
        const uint32_t ns = (uint32_t)t.n[s], q = rho / ns;
        K = key_add(K, tl[t.toff[s] + (rho - q * ns)], J);
        rho = q;
      }
    };
    int64_t sl = wa, base = 0;
    uint32_t e = (uint32_t)lane, K = 0;
    while (e >= S) {
      e -= S;
      ++sl;
    }
    if (sl < we) locate(sl, base, K);
    for (int64_t m0 = 0; m0 < tot; m0 += 64 * U) {
      float x[U];
      uint32_t pe[U], kk[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ok[u] = sl < we;
        x[u] = ok[u] ? __builtin_nontemporal_load(Xg + base + e) : 0.0f;
        pe[u] = e;
        kk[u] = K;
        e += 64;
        if (e >= S) {   // into the next slab (several when S < 64)
          do {
            e -= S;
            ++sl;
          } while (e >= S);
          if (sl < we) locate(sl, base, K);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) {
          const uint32_t pk = P[pe[u]];
          uint32_t bk = (pk & TT_KEY_MASK) + (kk[u] & TT_KEY_MASK);
          bk = bk >= J ? bk - J : bk;
          atomicAdd(&acc[bk], signed_f64(x[u], (pk ^ kk[u]) & TT_KEY_SIGN));
        }
    }
    __syncthreads();
    const int64_t gc = cpre[j] + c;
    const int64_t slot = w - owner(fpre[j] + c * F, W, Ttot);
    double* out = part + (spre[gc] + slot) * (int64_t)Jmax;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) out[b] = acc[b];
    __syncthreads();
    g = fpre[j] + c * F + qe;
  }
}

// k >= 2, key-sorted slabs: the units, partials and LDS tables of
// k_bsketch_slab, but slab q of a column is entry q of the problem's mode-k
// slab list, sorted by the key K over the modes other than 0, 1 and k.  A
// slab is read whole (V-value vectors when n_0 n_1 and the address of X
// allow it) by a group of TPI lanes (64, 128 or 256, the fewest that cover a
// piece of 256 MV vectors with MV = min(MS / V, 8) per lane), U slabs per
// load batch; the 256 / TPI groups split the workgroup's share of the list.  A group keeps FP64
// running sums of its slabs' entries while K stays the same and adds them
// to the accumulator at bucket P[e] + K when it changes: one LDS atomic per
// entry of a run of equal keys instead of one per entry of X.
template <int MS, int U>
__global__ __launch_bounds__(256) void k_bsketch_ks(const BTensor* __restrict__ T, const int32_t* __restrict__ tids,
                                                    const int64_t* __restrict__ fpre, const int64_t* __restrict__ cpre,
                                                    const int64_t* __restrict__ spre, int32_t nt, int32_t k,
                                                    double* __restrict__ part, int32_t Jmax, int32_t Smax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  uint32_t* P = reinterpret_cast<uint32_t*>(acc + Jmax);   // Smax entries
  uint32_t* tl = P + Smax;                                  // the problem's packed tables
  const int64_t W = gridDim.x, w = blockIdx.x;
  const int64_t Ttot = fpre[nt];
  const int64_t gs = w * Ttot / W, ge = (w + 1) * Ttot / W;
  if (gs >= ge) return;
  int j = seg_of(fpre, nt, gs), jp = -1;
  int64_t g = gs;
  while (g < ge) {
    while (fpre[j + 1] <= g) ++j;
    const BTensor& t = T[tids[j]];
    const int d = t.d;
    const uint32_t n0 = (uint32_t)t.n[0], n1 = (uint32_t)t.n[1];
    const uint32_t S = n0 * n1;
    const uint32_t J = t.J;
    int64_t Mp = 1, R = 1;
    for (int s = 2; s < k; ++s) Mp *= t.n[s];
    for (int s = k + 1; s < d; ++s) R *= t.n[s];
    const int64_t F = Mp * R;   // slabs per column
    const int64_t q0 = g - fpre[j];
    const int64_t c = q0 / F;
    const int64_t qa = q0 - c * F;
    const int64_t lim = ge - fpre[j] - c * F;
    const int64_t qe = lim < F ? lim : F;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) acc[b] = 0.0;
    if (j != jp) {   // P of a new problem (no thread reads it here)
      const int ntab = t.toff[1] + t.n[1];
      for (int i = threadIdx.x; i < ntab; i += blockDim.x) tl[i] = t.tab[i];
      __syncthreads();
      for (uint32_t e = threadIdx.x; e < S; e += blockDim.x) {
        const uint32_t i1 = e / n0;
        P[e] = key_add(tl[t.toff[0] + (e - i1 * n0)], tl[t.toff[1] + i1], J);
      }
      jp = j;
    }
    __syncthreads();
    // list entries {offset | sign, key} read as one 64-bit global load (x in the low half)
    typedef const uint64_t __attribute__((address_space(1)))* gu64;
    const gu64 lst = (gu64)t.sl[k];
    const int64_t cM = c * Mp;
    const uintptr_t xa = (uintptr_t)t.X;
    const int vw = (S % 4 == 0 && xa % 16 == 0) ? 4 : (S % 2 == 0 && xa % 8 == 0) ? 2 : 1;
    auto run_v = [&](auto Vc) {
      constexpr int V = decltype(Vc)::value;
      constexpr int MV = MS / V < 8 ? MS / V : 8;   // at most 8 vectors per lane: registers
      typedef typename FVec<V>::T vt;
      typedef const vt __attribute__((address_space(1)))* gvt;   // global loads: off the LDS wait counter
      const gvt Xv = (gvt)t.X;
      const uint32_t Sv = S / V;
      const int tpi = Sv <= 64u * MV ? 64 : Sv <= 128u * MV ? 128 : 256;
      const int ipw = 256 / tpi;
      const int grp = threadIdx.x / tpi, li = threadIdx.x - grp * tpi;
      for (uint32_t p0 = 0; p0 < Sv; p0 += (uint32_t)tpi * MV) {
        const int plen = (int)(Sv - p0 < (uint32_t)tpi * MV ? Sv - p0 : (uint32_t)tpi * MV);
        const int ms = (plen + tpi - 1) / tpi;
        double run[MV][V];
#pragma unroll
        for (int m = 0; m < MV; ++m)
#pragma unroll
          for (int i = 0; i < V; ++i) run[m][i] = 0.0;
        uint32_t cur = 0xffffffffu;   // key of the running sums (none yet)
        auto flush = [&]() {
#pragma unroll
          for (int m = 0; m < MV; ++m)
            if (m < ms && li + tpi * m < plen)
#pragma unroll
              for (int i = 0; i < V; ++i) {
                const uint32_t pk = P[(p0 + li + tpi * m) * V + i];
                uint32_t bk = (pk & TT_KEY_MASK) + cur;
                bk = bk >= J ? bk - J : bk;
                atomicAdd(&acc[bk], (pk & TT_KEY_SIGN) ? -run[m][i] : run[m][i]);
              }
#pragma unroll
          for (int m = 0; m < MV; ++m)
#pragma unroll
            for (int i = 0; i < V; ++i) run[m][i] = 0.0;
        };
        for (int64_t e0 = qa + grp; e0 < qe; e0 += (int64_t)ipw * U) {
          vt x[U][MV];
          uint32_t ky[U], sg[U];
          bool ok[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {   // all loads first, then the sums
            const int64_t e = e0 + (int64_t)ipw * u;
            ok[u] = e < qe;
            const uint64_t it = ok[u] ? lst[e] : 0ull;
            const uint32_t ix = (uint32_t)it;
            ky[u] = (uint32_t)(it >> 32);
            sg[u] = ix & TT_KEY_SIGN;
            const gvt base = Xv + ((int64_t)(ix & TT_KEY_MASK) + cM) * Sv + p0 + li;
#pragma unroll
            for (int m = 0; m < MV; ++m)
              x[u][m] = (ok[u] && m < ms && li + tpi * m < plen) ? base[tpi * m]
                                                                 : (vt)(0.0f);
          }
#pragma unroll
          for (int u = 0; u < U; ++u)   // in list order
            if (ok[u]) {
              if (ky[u] != cur) {
                if (cur != 0xffffffffu) flush();
                cur = ky[u];
              }
#pragma unroll
              for (int m = 0; m < MV; ++m)
#pragma unroll
                for (int i = 0; i < V; ++i) run[m][i] += signed_f64(lane_of<V>(x[u][m], i), sg[u]);
            }
        }
        if (cur != 0xffffffffu) flush();
      }
    };
    if (vw == 4) run_v(std::integral_constant<int, 4>());
    else if (vw == 2) run_v(std::integral_constant<int, 2>());
    else run_v(std::integral_constant<int, 1>());
    __syncthreads();
    const int64_t gc = cpre[j] + c;
    const int64_t slot = w - owner(fpre[j] + c * F, W, Ttot);
    double* out = part + (spre[gc] + slot) * (int64_t)Jmax;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) out[b] = acc[b];
    __syncthreads();
    g = fpre[j] + c * F + qe;
  }
}

// Y_j[b + J c] = sum over the partials of column (j, c), in slot order
// (units: slabs for the slab launch, else fibres).
__global__ void k_breduce(const BTensor* __restrict__ T, const int32_t* __restrict__ tids,
                          const int64_t* __restrict__ fpre, const int64_t* __restrict__ cpre,
                          const int64_t* __restrict__ spre, int32_t nt, int32_t k, const double* __restrict__ part,
                          int32_t Jmax, int64_t W, int32_t slab) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ncol = cpre[nt];
  if (idx >= ncol * Jmax) return;
  const int64_t gc = idx / Jmax;
  const uint32_t b = (uint32_t)(idx - gc * Jmax);
  const int j = seg_of(cpre, nt, gc);
  const BTensor& t = T[tids[j]];
  if (b >= t.J) return;
  const int64_t c = gc - cpre[j];
  int64_t F = 1;
  for (int s = slab ? 2 : 1; s < t.d; ++s)   // units of the launch: slabs or fibres
    if (s != k) F *= t.n[s];
  const int64_t Ttot = fpre[nt];
  const int64_t first = fpre[j] + c * F;
  const int64_t cnt = owner(first + F - 1, W, Ttot) - owner(first, W, Ttot) + 1;
  const double* p = part + spre[gc] * (int64_t)Jmax + b;
  double s = 0.0;
  for (int64_t q = 0; q < cnt; ++q) s += p[q * Jmax];
  t.Y[(int64_t)t.J * t.toff[k] + b + (int64_t)t.J * c] = (float)s;
}

// ---------------------------------------------------------------- k = 0
// Row b of Y_0: every fibre (i_1, o) whose key h_1(i_1) + h(o) is b adds its
// n_0 values with the signs of i_1 and o.  The outer tuples o of a key are a
// contiguous range of the problem's bucket-sorted list, so the fibres of row
// i_1 are those of key b - h_1(i_1).  The workgroup finds the ranges of 256
// rows at once (a thread per row, then a prefix sum of their lengths in LDS);
// the fibres of those rows then form one sequence split over all lane
// groups, FIB fibres per group per load batch.  A problem whose k = 0 step
// wrote the outer sketch (zo set) reads that sketch in place of X, with one
// "tuple" per key: its row r of the sketch, outer signs already applied.
template <int NJ, int FIB>
__global__ __launch_bounds__(256) void k_bsketch_0(const BTensor* __restrict__ T, const int32_t* __restrict__ tids,
                                                   int32_t Jmax) {
  __shared__ double red[4][64 * NJ];
  __shared__ int64_t rpre[257];   // fibres of the chunk's rows before row q
  __shared__ uint32_t rbeg[256];  // list position of row q's first fibre
  __shared__ uint32_t rsg[256];   // sign of i_1 of row q
  __shared__ int64_t wsum[4];
  const int j = blockIdx.x / Jmax;
  const uint32_t b = blockIdx.x - (uint32_t)j * Jmax;
  const BTensor& t = T[tids[j]];
  if (b >= t.J) return;
  const bool oz = t.zo != nullptr;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n0 = t.n[0], n1 = t.n[1];
  const uint32_t J = t.J;
  const int lpf_log2 = lpf_log2_of<NJ>(n0);
  const int LPF = 1 << lpf_log2, G = 64 >> lpf_log2;
  const int gi = lane >> lpf_log2, v = lane & (LPF - 1);
  const int ng = 4 * G, gid = wv * G + gi;   // lane groups of the workgroup
  const uint32_t* tab1 = t.tab + t.toff[1];
  const gfloat Xg = (gfloat)(oz ? t.zo : t.X);
  const guint offg = (guint)t.off, sortg = (guint)t.sorted;
  double acc[NJ];   // FP64: the result does not depend on the order of the fibres
#pragma unroll
  for (int q = 0; q < NJ; ++q) acc[q] = 0.0;
  for (int r0 = 0; r0 < n1; r0 += 256) {
    const int nr = n1 - r0 < 256 ? n1 - r0 : 256;
    const int i1 = r0 + (int)threadIdx.x;
    int64_t cnt = 0;
    uint32_t bg = 0, sg = 0;
    if (i1 < n1) {
      const uint32_t t1 = tab1[i1], h1 = t1 & TT_KEY_MASK;
      const uint32_t c = b >= h1 ? b - h1 : b + J - h1;
      sg = t1 & TT_KEY_SIGN;
      if (oz) {
        bg = c;
        cnt = 1;
      } else {
        bg = offg[c];
        cnt = offg[c + 1] - bg;
      }
    }
    int64_t inc = cnt;   // inclusive prefix over the wave, then over the waves
    for (int m = 1; m < 64; m <<= 1) {
      const int64_t o = __shfl_up(inc, m, 64);
      if (lane >= m) inc += o;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    for (int w = 0; w < wv; ++w) inc += wsum[w];
    rpre[threadIdx.x + 1] = inc;
    if (threadIdx.x == 0) rpre[0] = 0;
    rbeg[threadIdx.x] = bg;
    rsg[threadIdx.x] = sg;
    __syncthreads();
    const int64_t tot = rpre[nr];
    for (int64_t f0 = 0; f0 < tot; f0 += (int64_t)ng * FIB) {
      float x[FIB][NJ];
      uint32_t sgn[FIB];
#pragma unroll
      for (int u = 0; u < FIB; ++u) {   // all loads first, then the sums
        const int64_t f = f0 + (int64_t)u * ng + gid;
        const bool ok = f < tot;
        int lo = 0, hi = nr - 1;   // the row of fibre f: the last q with rpre[q] <= f
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (rpre[mid] <= f) lo = mid;
          else hi = mid - 1;
        }
        const uint32_t pos = rbeg[lo] + (uint32_t)(f - rpre[lo]);
        const uint32_t item = !ok ? 0u : oz ? pos : sortg[pos];
        sgn[u] = (item ^ rsg[lo]) & TT_KEY_SIGN;
        const gfloat base = Xg + ((int64_t)(item & TT_KEY_MASK) * n1 + r0 + lo) * (int64_t)n0;
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
          const int i0 = v + LPF * q;
          x[u][q] = (ok && i0 < n0) ? __builtin_nontemporal_load(base + i0) : 0.0f;
        }
      }
#pragma unroll
      for (int u = 0; u < FIB; ++u)
#pragma unroll
        for (int q = 0; q < NJ; ++q) acc[q] += signed_f64(x[u][q], sgn[u]);
    }
    __syncthreads();   // the next chunk rewrites the row arrays
  }
  for (int m = LPF; m < 64; m <<= 1)
#pragma unroll
    for (int q = 0; q < NJ; ++q) acc[q] += __shfl_xor(acc[q], m, 64);
  if (gi == 0)
#pragma unroll
    for (int q = 0; q < NJ; ++q) red[wv][v + LPF * q] = acc[q];
  __syncthreads();
  for (int i = threadIdx.x; i < n0; i += blockDim.x) {
    double s = 0.0;
    for (int ww = 0; ww < 4; ++ww) s += red[ww][i];
    t.Y[b + (int64_t)J * i] = (float)s;
  }
}

constexpr int kZoMS = 16, kZoU = 2;   // FP32 entries per lane of a slab piece, slabs per load batch

// k = 0 of the problems whose Y_1 comes from the outer sketch: workgroup
// (f, c) adds the contiguous n_0 x n_1 slabs of the outer tuples hashed to
// bucket c, each with its outer sign, into zo[c n_0 n_1 + i_1 n_0 + i_0].
// Each slab is read by one workgroup, so no 128-byte line is fetched twice
// except where two slabs meet.  A slab is read in V-entry vectors (V = 4 or
// 2 when n_0 n_1 and the address of X allow it: every slab then starts on a
// V-entry boundary) and taken in pieces of at most 256 MS entries; a group
// of TPI lanes (64, 128 or 256, the fewest that cover a piece with MS
// entries per lane) sums one slab of the bucket at a time in FP64 registers,
// U slabs per load batch, the 256 / TPI groups splitting the bucket's list;
// the groups are then added in a fixed order.  fids lists the problems of
// this V.  Plain (L2-allocating) loads: the lines that two consecutive load
// instructions of a group share are then fetched once (non-temporal loads
// fetched them twice for 1- and 2-value vectors).
template <int V, int MS, int U>
__global__ __launch_bounds__(256) void kb_zo(const BTensor* __restrict__ T, const int32_t* __restrict__ fids,
                                             int32_t Jmax) {
  typedef typename FVec<V>::T vt;
  constexpr int MV = MS / V;              // vectors per lane of a piece
  __shared__ double red[3 * 64 * MS];     // groups 1..3 (TPI = 64) or group 1 (TPI = 128)
  const int f = blockIdx.x / Jmax;
  const uint32_t c = blockIdx.x - (uint32_t)f * Jmax;
  const BTensor& t = T[fids[f]];
  if (c >= t.J) return;
  const int64_t Sv = (int64_t)t.n[0] * t.n[1] / V;   // vectors per slab
  const int tpi = Sv <= 64 * MV ? 64 : Sv <= 128 * MV ? 128 : 256;
  const int ipw = 256 / tpi;
  const int grp = threadIdx.x / tpi, li = threadIdx.x - grp * tpi;
  const guint offg = (guint)t.off, sortg = (guint)t.sorted;
  const uint32_t beg = offg[c], end = offg[c + 1];
  typedef const vt __attribute__((address_space(1)))* gvt;
  const gvt Xv = (gvt)t.X;
  vt* zo = reinterpret_cast<vt*>(t.zo) + (int64_t)c * Sv;
  for (int64_t p0 = 0; p0 < Sv; p0 += (int64_t)tpi * MV) {
    const int plen = (int)(Sv - p0 < (int64_t)tpi * MV ? Sv - p0 : (int64_t)tpi * MV);
    const int ms = (plen + tpi - 1) / tpi;
    double acc[MV][V];
#pragma unroll
    for (int m = 0; m < MV; ++m)
#pragma unroll
      for (int i = 0; i < V; ++i) acc[m][i] = 0.0;
    for (uint32_t e0 = beg + grp; e0 < end; e0 += ipw * U) {
      vt x[U][MV];
      uint32_t sg[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {   // all loads first, then the sums
        const uint32_t e = e0 + ipw * u;
        const bool ok = e < end;
        const uint32_t item = ok ? sortg[e] : 0u;
        sg[u] = item & TT_KEY_SIGN;
        const gvt base = Xv + (int64_t)(item & TT_KEY_MASK) * Sv + p0 + li;
#pragma unroll
        for (int m = 0; m < MV; ++m)
          x[u][m] = (ok && m < ms && li + tpi * m < plen) ? base[tpi * m] : (vt)(0.0f);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)   // in list order
#pragma unroll
        for (int m = 0; m < MV; ++m)
#pragma unroll
          for (int i = 0; i < V; ++i) acc[m][i] += signed_f64(lane_of<V>(x[u][m], i), sg[u]);
    }
    if (ipw > 1) {
      __syncthreads();   // the previous piece's reads of red are done
      if (grp > 0)
#pragma unroll
        for (int m = 0; m < MV; ++m)
          if (m < ms)
#pragma unroll
            for (int i = 0; i < V; ++i) red[((grp - 1) * tpi * MV + li + tpi * m) * V + i] = acc[m][i];
      __syncthreads();
      if (grp == 0)
        for (int g = 1; g < ipw; ++g)
#pragma unroll
          for (int m = 0; m < MV; ++m)
            if (m < ms)
#pragma unroll
              for (int i = 0; i < V; ++i) acc[m][i] += red[((g - 1) * tpi * MV + li + tpi * m) * V + i];
    }
    if (grp == 0)
#pragma unroll
      for (int m = 0; m < MV; ++m)
        if (m < ms && li + tpi * m < plen) {
          vt o;
          if constexpr (V == 1) {
            o = (float)acc[m][0];
          } else {
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = (float)acc[m][i];
          }
          zo[p0 + li + tpi * m] = o;
        }
  }
}

// Y_1 of a problem whose k = 0 step wrote its outer sketch: workgroup
// (i_1, f) adds row (r, i_1) of the sketch (outer key r) at bucket
// r + h_0(i_0) with the sign of i_0, in a J-entry FP64 LDS array, and writes
// column i_1 of Y_1.
__global__ __launch_bounds__(256) void kb_y1_outer(const BTensor* __restrict__ T, const int32_t* __restrict__ fids) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const BTensor& t = T[fids[blockIdx.y]];
  const int i1 = blockIdx.x;
  const int n0 = t.n[0];
  if (i1 >= t.n[1]) return;
  const uint32_t J = t.J;
  double* acc = reinterpret_cast<double*>(smem_raw);
  uint32_t* t0 = reinterpret_cast<uint32_t*>(acc + J);
  for (uint32_t q = threadIdx.x; q < J; q += blockDim.x) acc[q] = 0.0;
  for (int q = threadIdx.x; q < n0; q += blockDim.x) t0[q] = t.tab[t.toff[0] + q];
  __syncthreads();
  const int64_t n1 = t.n[1];
  const uint32_t tot = J * (uint32_t)n0;
  for (uint32_t q = threadIdx.x; q < tot; q += blockDim.x) {
    const uint32_t r = q / (uint32_t)n0, i0 = q - r * (uint32_t)n0;
    const uint32_t tv = t0[i0];
    uint32_t bk = r + (tv & TT_KEY_MASK);
    bk = bk >= J ? bk - J : bk;
    atomicAdd(&acc[bk], signed_f64(t.zo[((int64_t)r * n1 + i1) * n0 + i0], tv & TT_KEY_SIGN));
  }
  __syncthreads();
  float* y = t.Y + (int64_t)J * t.toff[1] + (int64_t)J * i1;
  for (uint32_t q = threadIdx.x; q < J; q += blockDim.x) y[q] = (float)acc[q];
}

__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (threadIdx.x == 0) p[0] = v;
}
__global__ void k_inc_i64(int64_t* p) {
  if (threadIdx.x == 0) p[0] += 1;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

typedef void (*BKFn)(const BTensor*, const int32_t*, const int64_t*, const int64_t*, const int64_t*, int32_t, int32_t,
                     double*, int32_t);
typedef void (*B0Fn)(const BTensor*, const int32_t*, int32_t);

// the compiled (entries per lane, fibres in flight) shapes
BKFn bk_kernel(int nj, int fib) {
  if (nj == 2) return fib == 8 ? k_bsketch_k<2, 8> : k_bsketch_k<2, 16>;
  return fib == 8 ? k_bsketch_k<4, 8> : k_bsketch_k<4, 16>;
}
typedef void (*BSFn)(const BTensor*, const int32_t*, const int64_t*, const int64_t*, const int64_t*, int32_t, int32_t,
                     double*, int32_t, int32_t);
// slab steps: 4 or 8 rows in flight of the stream in memory order, or 1 or 2
// slabs per group in flight of the key-sorted stream
BSFn bs_kernel(int rows) {
  return rows == 1 ? k_bsketch_ks<16, 1> : rows == 2 ? k_bsketch_ks<16, 2> : rows == 4 ? k_bsketch_slab<4>
                                                                                      : k_bsketch_slab<8>;
}
bool slab_sorted(int rows) { return rows <= 2; }

B0Fn b0_kernel(int nj, int fib) {
  if (nj == 2) return fib == 4 ? k_bsketch_0<2, 4> : k_bsketch_0<2, 8>;
  return fib == 4 ? k_bsketch_0<4, 4> : k_bsketch_0<4, 8>;
}

}  // namespace

struct tt_batch_s {
  int32_t count = 0;
  std::vector<tt_plan> plans;
  std::vector<size_t> plan_off;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_need = 0;
  int max_d = 0;
  int32_t Jmax = 0;
  int max_n0 = 1;
  // tuning per step k: entries per lane and fibres in flight of the data
  // sketch, Gram K-chunk of the core updates (the workgroup count is W below)
  int nj[TT_MAX_ORDER] = {}, fib[TT_MAX_ORDER] = {};
  int32_t kchunk[TT_MAX_ORDER] = {};
  // per step k: problems of order > k (core updates), and the problems whose
  // data sketch the step's launch covers with their unit prefixes (at k = 1
  // the problems in fids are left out: their Y_1 comes from the outer sketch
  // of the k = 0 step)
  std::vector<std::vector<int32_t>> tids, stids;
  std::vector<std::vector<int64_t>> fpre, cpre, spre;
  std::vector<int32_t> fids;
  size_t o_fids = 0;
  // the problems of fids by the load width of their outer-sketch pass (4, 2,
  // 1 FP32 values), set with the X pointers: counts and the device list
  int32_t zcnt[3] = {};
  size_t o_zids = 0;
  int32_t fid_n1 = 0;          // largest n_1 among fids
  size_t o_desc = 0, o_part = 0, o_counter = 0;
  // the key sorts of step k, one launch set for all its problems (k = 0: the
  // outer tuples; k >= 2 on the slab path: the slabs of a mode-k column, for
  // the key-sorted slab kernel): argument sets and (set, chunk) per workgroup
  size_t o_sargs[TT_MAX_ORDER] = {}, o_ssrc[TT_MAX_ORDER] = {};
  int32_t sort_sets[TT_MAX_ORDER] = {}, sort_blocks[TT_MAX_ORDER] = {};
  // slab steps whose slab offsets fit the key sort (the key-sorted kernel is
  // then among the tuner's choices)
  bool ssort[TT_MAX_ORDER] = {};
  // batched core updates per step k: descriptors, QR classes, launch bounds
  struct QrClass {
    int32_t rmax, rpt, off, cnt;
  };
  std::vector<std::vector<BUpd>> upd;
  std::vector<std::vector<QrClass>> qcls;
  std::vector<std::vector<int32_t>> qidx, qfall;   // QR class members (index into upd[k]); per-problem QRs
  size_t o_upd[TT_MAX_ORDER] = {}, o_qidx[TT_MAX_ORDER] = {};
  // batched right-to-left orthogonalisation, per step s >= 1 (problems of
  // order > s): descriptors, QR classes, per-problem QRs, largest G_{s-1}
  // row count; columns of the sweep-start core transforms
  std::vector<std::vector<BRo>> ro;
  std::vector<std::vector<QrClass>> rcls;
  std::vector<std::vector<int32_t>> ridx, rids, rfall;
  size_t o_ro[TT_MAX_ORDER] = {}, o_ridx[TT_MAX_ORDER] = {};
  int32_t ro_rows[TT_MAX_ORDER] = {};
  int32_t fft0_cols = 0;
  // batched table generation: argument sets (device), largest table
  size_t o_tabargs = 0;
  int64_t tab_max = 0;
  // batched interface of each step: descriptors, largest core-transform and
  // output column counts, waves of a chain workgroup
  std::vector<std::vector<BIface>> bif;
  size_t o_bif[TT_MAX_ORDER] = {};
  int32_t if_cols[TT_MAX_ORDER] = {}, if_s[TT_MAX_ORDER] = {};
  int32_t if_cw = 1;
  int32_t g_gx[TT_MAX_ORDER] = {}, g_count[TT_MAX_ORDER] = {}, g_cbb[TT_MAX_ORDER] = {}, g_cols[TT_MAX_ORDER] = {};
  size_t g_lchol[TT_MAX_ORDER] = {}, g_ltrsm[TT_MAX_ORDER] = {};
  std::vector<const void*> upd_key;
  hipEvent_t ev_main = nullptr;
  size_t o_tids[TT_MAX_ORDER], o_stids[TT_MAX_ORDER], o_fpre[TT_MAX_ORDER], o_cpre[TT_MAX_ORDER],
      o_spre[TT_MAX_ORDER];
  int64_t Wmax = 16384;
  int64_t W[TT_MAX_ORDER];   // workgroups of the k >= 1 launch (0: device occupancy)
  // k >= 2 steps run in slab units when every slab and table set fits in LDS
  bool slab[TT_MAX_ORDER] = {};
  int32_t slab_S[TT_MAX_ORDER] = {}, slab_tab[TT_MAX_ORDER] = {};
  // descriptors as last uploaded
  std::vector<BTensor> host_desc;
  bool desc_valid = false;
  // graph
  bool use_graph = false;
  hipStream_t cap = nullptr;   // private stream the sweep is captured on
  hipStream_t side = nullptr;  // batched data sketches of a sweep
  hipStream_t lane[8] = {};    // per-problem orthogonalisation and tables
  hipEvent_t ev_fork = nullptr, ev_done = nullptr, ev_lane[8] = {}, ev_step[TT_MAX_ORDER] = {};
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> cap_ptrs;
  int64_t replays = 0;
};

namespace {

size_t step_lds(tt_batch b, int k) {
  return sizeof(double) * b->Jmax + (b->slab[k] ? sizeof(uint32_t) * (size_t)(b->slab_S[k] + b->slab_tab[k]) : 0);
}

// resident workgroups of the step-k launch on the whole device
int occupancy_grid(tt_batch b, int k, int nj, int fib) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    ncu = 256;
  const size_t lds = step_lds(b, k);
  hipError_t e = hipErrorInvalidValue;
  if (b->slab[k]) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bs_kernel(fib), 256, lds);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bk_kernel(nj, fib), 256, lds);
  if (e != hipSuccess || per < 1) per = 1;
  return per * ncu;
}

std::vector<const void*> pointer_key(tt_batch b, const void* const* X, void* const* const* cores) {
  std::vector<const void*> key;
  for (int i = 0; i < b->count; ++i) {
    key.push_back(X[i]);
    for (int s = 0; s < b->plans[i]->d; ++s) key.push_back(cores[i][s]);
  }
  return key;
}

tt_status check_inputs(tt_batch b, const void* const* X, void* const* const* cores) {
  if (!X || !cores) return tt_fail(TT_ERR_ARG, "null X or core arrays");
  for (int i = 0; i < b->count; ++i) {
    if (!X[i] || !cores[i]) return tt_fail(TT_ERR_ARG, "problem %d: null X or cores", i);
    for (int s = 0; s < b->plans[i]->d; ++s)
      if (!cores[i][s]) return tt_fail(TT_ERR_ARG, "problem %d: core %d is null", i, s);
  }
  return TT_OK;
}

// upload the per-problem descriptors (X pointers may change between calls)
tt_status upload_desc(tt_batch b, const void* const* X) {
  bool same = b->desc_valid;
  for (int i = 0; i < b->count && same; ++i) same = b->host_desc[i].X == X[i];
  if (same) return TT_OK;
  for (int i = 0; i < b->count; ++i) {
    tt_plan p = b->plans[i];
    BTensor& t = b->host_desc[i];
    t.X = static_cast<const float*>(X[i]);
    t.Y = p->at<float>(p->o_Yall);
    t.tab = p->at<uint32_t>(p->o_tab);
    t.off = p->at<uint32_t>(p->o_cnt);
    t.sorted = p->at<uint32_t>(p->o_sortO);
    t.zo = tt_sketch_fused01(p) ? p->at<float>(p->o_zo) : nullptr;
    for (int s = 0; s < TT_MAX_ORDER; ++s) t.sl[s] = s >= 2 && s < p->d ? tt_fibre_list(p, s) : nullptr;
    for (int s = 0; s < TT_MAX_ORDER; ++s) {
      t.n[s] = s < p->d ? (int32_t)p->n[s] : 1;
      t.toff[s] = s < p->d ? (int32_t)p->tab_off[s] : 0;
    }
    t.d = p->d;
    t.J = (uint32_t)p->J;
  }
  TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_desc, b->host_desc.data(), sizeof(BTensor) * b->count, hipMemcpyHostToDevice,
                            b->stream));
  // outer-sketch problems by load width: V-entry vectors need n_0 n_1 and the
  // address of X divisible by V (largest slabs first within each width)
  std::vector<int32_t> zids;
  for (int vc = 0; vc < 3; ++vc) {
    const int V = 4 >> vc;
    b->zcnt[vc] = 0;
    for (int32_t i : b->fids) {
      const int64_t S = b->plans[i]->n[0] * b->plans[i]->n[1];
      const uintptr_t a = (uintptr_t)X[i];
      const int w = (S % 4 == 0 && a % 16 == 0) ? 4 : (S % 2 == 0 && a % 8 == 0) ? 2 : 1;
      if (w != V) continue;
      zids.push_back(i);
      b->zcnt[vc] += 1;
    }
  }
  if (!zids.empty())
    TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_zids, zids.data(), sizeof(int32_t) * zids.size(), hipMemcpyHostToDevice,
                              b->stream));
  TT_HIP_TRY(hipStreamSynchronize(b->stream));
  b->desc_valid = true;
  return TT_OK;
}

hipError_t launch_step_sketch(tt_batch b, int k, int64_t Wk) {
  const BTensor* T = reinterpret_cast<const BTensor*>(b->ws + b->o_desc);
  const int32_t* tids = reinterpret_cast<const int32_t*>(b->ws + b->o_stids[k]);
  const int32_t nt = (int32_t)b->stids[k].size();
  hipError_t e;
  if (k == 1 && !b->fids.empty()) {
    // Y_1 of the problems whose step-0 launch wrote the outer sketch (the
    // launch of step 0 precedes this one on the stream)
    const size_t lds = sizeof(double) * b->Jmax + sizeof(uint32_t) * b->max_n0;
    if ((e = tt_allow_lds(kb_y1_outer, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(kb_y1_outer, dim3((unsigned)b->fid_n1, (unsigned)b->fids.size()), dim3(256), lds, b->stream, T,
                       reinterpret_cast<const int32_t*>(b->ws + b->o_fids));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (k == 0) {
    if (b->sort_sets[0] > 0 &&
        (e = launch_outer_sorts_batched(b->ws + b->o_sargs[0], b->ws + b->o_ssrc[0], b->sort_sets[0],
                                        b->sort_blocks[0], b->Jmax, b->stream)) != hipSuccess)
      return e;
    // the outer sketch, which Y_0 of those problems then reads: one launch per load width
    const int32_t* zids = reinterpret_cast<const int32_t*>(b->ws + b->o_zids);
    for (int vc = 0, at = 0; vc < 3; at += b->zcnt[vc], ++vc) {
      if (b->zcnt[vc] == 0) continue;
      const dim3 gz((unsigned)b->zcnt[vc] * (unsigned)b->Jmax);
      if (vc == 0) hipLaunchKernelGGL((kb_zo<4, kZoMS, kZoU>), gz, dim3(256), 0, b->stream, T, zids + at, b->Jmax);
      else if (vc == 1) hipLaunchKernelGGL((kb_zo<2, kZoMS, kZoU>), gz, dim3(256), 0, b->stream, T, zids + at, b->Jmax);
      else hipLaunchKernelGGL((kb_zo<1, kZoMS, kZoU>), gz, dim3(256), 0, b->stream, T, zids + at, b->Jmax);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (nt == 0) return hipSuccess;
    const dim3 grid((unsigned)(nt * b->Jmax));
    hipLaunchKernelGGL(b0_kernel(b->nj[0], b->fib[0]), grid, dim3(256), 0, b->stream, T, tids, b->Jmax);
    return hipGetLastError();
  }
  if (nt == 0) return hipSuccess;
  const int64_t* fpre = reinterpret_cast<const int64_t*>(b->ws + b->o_fpre[k]);
  const int64_t* cpre = reinterpret_cast<const int64_t*>(b->ws + b->o_cpre[k]);
  const int64_t* spre = reinterpret_cast<const int64_t*>(b->ws + b->o_spre[k]);
  double* part = reinterpret_cast<double*>(b->ws + b->o_part);
  const int64_t Ttot = b->fpre[k].back();
  int64_t W = Wk > 0 ? Wk : occupancy_grid(b, k, b->nj[k], b->fib[k]);
  if (W > b->Wmax) W = b->Wmax;
  if (W > Ttot) W = Ttot;
  if (W < 1) W = 1;
  const size_t lds = step_lds(b, k);
  if (b->slab[k] && slab_sorted(b->fib[k]) &&
      (e = launch_outer_sorts_batched(b->ws + b->o_sargs[k], b->ws + b->o_ssrc[k], b->sort_sets[k], b->sort_blocks[k],
                                      b->Jmax, b->stream)) != hipSuccess)
    return e;
  if (b->slab[k])
    hipLaunchKernelGGL(bs_kernel(b->fib[k]), dim3((unsigned)W), dim3(256), lds, b->stream, T, tids, fpre, cpre, spre, nt,
                       k, part, b->Jmax, b->slab_S[k]);
  else
    hipLaunchKernelGGL(bk_kernel(b->nj[k], b->fib[k]), dim3((unsigned)W), dim3(256), lds, b->stream, T, tids, fpre,
                       cpre, spre, nt, k, part, b->Jmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t total = b->cpre[k].back() * b->Jmax;
  hipLaunchKernelGGL(k_breduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, b->stream, T, tids, fpre, cpre,
                     spre, nt, k, part, b->Jmax, W, b->slab[k] ? 1 : 0);
  return hipGetLastError();
}

constexpr int kLanes = 8;   // streams the per-problem core updates are spread over

tt_status make_lanes(tt_batch b) {
  if (b->side) return TT_OK;
  TT_HIP_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
  for (int l = 0; l < kLanes; ++l) {
    TT_HIP_TRY(hipStreamCreateWithFlags(&b->lane[l], hipStreamNonBlocking));
    TT_HIP_TRY(hipEventCreateWithFlags(&b->ev_lane[l], hipEventDisableTiming));
  }
  TT_HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
  TT_HIP_TRY(hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
  TT_HIP_TRY(hipEventCreateWithFlags(&b->ev_main, hipEventDisableTiming));
  for (int k = 0; k < TT_MAX_ORDER; ++k) TT_HIP_TRY(hipEventCreateWithFlags(&b->ev_step[k], hipEventDisableTiming));
  return TT_OK;
}

// Fill and upload the core-update descriptors (core pointers may change
// between calls; the descriptors live in device memory, so a captured graph
// stays valid when only their contents change).
// the plan-buffer pointers of the core-update descriptors (fixed once the
// workspace is bound)
void fill_upd_buffers(tt_batch b) {
  for (int k = 0; k < b->max_d; ++k)
    for (size_t j = 0; j < b->upd[k].size(); ++j) {
      tt_plan p = b->plans[b->tids[k][j]];
      BUpd& u = b->upd[k][j];
      u.SH = p->at<float>(p->o_SH);
      u.Y = p->at<float>(p->o_Yall) + p->J * p->tab_off[k];
      u.gpart = p->at<double>(p->o_gram);
      u.gsum = p->at<double>(p->o_gsum);
      u.Lg = p->at<double>(p->o_minv);
      u.status = p->at<int32_t>(p->o_status);
      u.R = p->at<double>(p->o_qrR);
    }
}

// Gram K-chunk of step k; the descriptors and the launch width follow, and
// the next sweep uploads them again
void set_kchunk(tt_batch b, int k, int32_t kc) {
  b->kchunk[k] = kc;
  int32_t gx = 0;
  for (BUpd& u : b->upd[k]) {
    u.kchunk = kc;
    u.chunks = (u.J + kc - 1) / kc;
    const int tiles = ((u.s + 15) / 16) * ((u.s + u.nk + 15) / 16);
    gx = std::max(gx, ((tiles + 3) / 4) * u.chunks);
  }
  b->g_gx[k] = gx;
  b->upd_key.clear();
}

tt_status upload_upd(tt_batch b, void* const* const* cores) {
  std::vector<const void*> key;
  for (int i = 0; i < b->count; ++i)
    for (int s2 = 0; s2 < b->plans[i]->d; ++s2) key.push_back(cores[i][s2]);
  if (key == b->upd_key) return TT_OK;
  for (int k = 0; k < b->max_d; ++k) {
    for (size_t j = 0; j < b->upd[k].size(); ++j) {
      const int i = b->tids[k][j];
      tt_plan p = b->plans[i];
      BUpd& u = b->upd[k][j];
      u.G = static_cast<double*>(cores[i][k]);
      const bool fall = std::find(b->qfall[k].begin(), b->qfall[k].end(), i) != b->qfall[k].end();
      u.Gnext = (k + 1 < p->d && !fall) ? static_cast<double*>(cores[i][k + 1]) : nullptr;
    }
    if (!b->upd[k].empty())
      TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_upd[k], b->upd[k].data(), sizeof(BUpd) * b->upd[k].size(),
                                hipMemcpyHostToDevice, b->stream));
    // the interface descriptors of step k
    b->bif[k].resize(b->tids[k].size());
    for (size_t j = 0; j < b->tids[k].size(); ++j) {
      const int i = b->tids[k][j];
      tt_plan p = b->plans[i];
      BIface& f = b->bif[k][j];
      f.cd = tt_make_desc(p, cores[i]);
      f.tab = p->at<uint32_t>(p->o_tab);
      f.chat = p->ws + p->o_chat;
      f.pre = p->ws + p->o_pre;
      f.suf = p->ws + p->o_suf;
      f.SH = p->ws + p->o_SH;
      f.tw = p->ws + p->o_tw;
      f.fft_code = 0;
      for (int r = 0; r < p->fft_nrad; ++r) f.fft_code |= (uint64_t)p->fft_radix[r] << (4 * r);
      f.fft_nrad = p->fft_nrad;
      f.J = (int32_t)p->J;
      f.k = k;
      f.cols = k >= 1 ? (int32_t)(p->r[k - 1] * p->r[k]) : 0;
      f.s = (int32_t)(p->r[k] * p->r[k + 1]);
    }
    if (!b->bif[k].empty())
      TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_bif[k], b->bif[k].data(), sizeof(BIface) * b->bif[k].size(),
                                hipMemcpyHostToDevice, b->stream));
  }
  for (int k = 1; k < b->max_d; ++k) {
    for (size_t j = 0; j < b->ro[k].size(); ++j) {
      const int i = b->rids[k][j];
      tt_plan p = b->plans[i];
      BRo& u = b->ro[k][j];
      u.G = static_cast<double*>(cores[i][k]);
      u.R = p->at<double>(p->o_qrR);
      const bool fall = std::find(b->rfall[k].begin(), b->rfall[k].end(), (int32_t)j) != b->rfall[k].end();
      u.Gprev = fall ? nullptr : static_cast<double*>(cores[i][k - 1]);
    }
    if (!b->ro[k].empty())
      TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_ro[k], b->ro[k].data(), sizeof(BRo) * b->ro[k].size(),
                                hipMemcpyHostToDevice, b->stream));
  }
  TT_HIP_TRY(hipStreamSynchronize(b->stream));
  b->upd_key = key;
  return TT_OK;
}

// Enqueue one sweep of every problem.  The batched data sketches of all steps
// need only X and the sweep's tables, so they go first, on the side stream,
// one launch per step.  On the batch stream: the right-to-left
// orthogonalisation, one step s at a time for every problem of order > s
// (QRs grouped by register shape, taller ones per problem, one absorb launch),
// and the transforms of cores 1..d-1 in one launch.  Then per step k: one
// launch per kernel computes the interface sketches (and the new transform of
// core k - 1) of every problem of order > k; then one launch each covers the
// Gram, the solve (summed partials, Cholesky, substitution) and the QR +
// absorb of every problem of order > k.  The next sweep's tables are drawn,
// in one launch, once every sketch has read the current ones.  Everything
// forks from and joins back into the batch stream.
tt_status enqueue_sweep(tt_batch b, void* const* const* cores) {
  tt_status st;
  if ((st = make_lanes(b))) return st;
  const hipStream_t main = b->stream;
  // the next sweep's tables: one launch for every problem unless a plan's
  // tables are overridden or its FFT roots still need filling (then per
  // problem, on lanes)
  bool tables_batched = b->o_tabargs != 0;
  for (tt_plan p : b->plans) tables_batched = tables_batched && !p->override_tables && p->tw_J == p->J;
  TT_HIP_TRY(hipEventRecord(b->ev_fork, main));
  TT_HIP_TRY(hipStreamWaitEvent(b->side, b->ev_fork, 0));
  if (!tables_batched)
    for (int l = 0; l < kLanes; ++l) TT_HIP_TRY(hipStreamWaitEvent(b->lane[l], b->ev_fork, 0));
  // data sketches
  b->stream = b->side;
  for (int k = 0; k < b->max_d; ++k) {
    const hipError_t e = launch_step_sketch(b, k, b->W[k]);
    if (e != hipSuccess) {
      b->stream = main;
      return tt_fail(TT_ERR_HIP, "batched sketch launch failed: %s", hipGetErrorString(e));
    }
    TT_HIP_TRY(hipEventRecord(b->ev_step[k], b->side));
  }
  hipLaunchKernelGGL(k_inc_i64, dim3(1), dim3(64), 0, b->side, reinterpret_cast<int64_t*>(b->ws + b->o_counter));
  TT_HIP_TRY(hipGetLastError());
  TT_HIP_TRY(hipEventRecord(b->ev_done, b->side));
  b->stream = main;
  std::vector<CoreDesc> cd(b->count);
  std::vector<hipStream_t> keep(b->count);
  for (int i = 0; i < b->count; ++i) {
    keep[i] = b->plans[i]->stream;
    cd[i] = tt_make_desc(b->plans[i], cores[i]);
  }
  auto lane_of = [&](int i) { return b->lane[i % kLanes]; };
  auto restore = [&]() {
    for (int i = 0; i < b->count; ++i) b->plans[i]->stream = keep[i];
  };
  // right-to-left orthogonalisation, one step s at a time for every problem
  // of order > s (register QRs by class, taller ones per problem, then the
  // absorb of R into core s - 1), and the transforms of cores 1..d-1
  for (int k = b->max_d - 1; k >= 1; --k) {
    const BRo* dr = reinterpret_cast<const BRo*>(b->ws + b->o_ro[k]);
    const int32_t* ix = reinterpret_cast<const int32_t*>(b->ws + b->o_ridx[k]);
    for (const auto& c : b->rcls[k]) TT_HIP_TRY(launch_qr_right_batched(dr, ix + c.off, c.cnt, c.rmax, c.rpt, main));
    for (int32_t j : b->rfall[k]) {
      const int i = b->rids[k][j];
      tt_plan p = b->plans[i];
      const BRo& u = b->ro[k][j];
      p->stream = main;
      double* const* G = reinterpret_cast<double* const*>(cores[i]);
      TT_HIP_TRY(launch_qr_core(p, G[k], u.m, u.r, u.r, 1));
      TT_HIP_TRY(launch_absorb_right(p, G[k - 1], u.rows, u.r));
      p->stream = keep[i];
    }
    TT_HIP_TRY(launch_absorb_right_batched(dr, (int32_t)b->ro[k].size(), b->ro_rows[k], main));
  }
  TT_HIP_TRY(launch_core_fft_batched(b->ws + b->o_bif[0], (int32_t)b->tids[0].size(), b->Jmax, b->fft0_cols, main));
  for (int k = 0; k < b->max_d; ++k) {
    const int32_t nt = (int32_t)b->tids[k].size();
    // the transform of core k - 1 (changed in step k - 1) and the interface
    // sketches of step k, one launch each for all problems of order > k
    {
      const hipError_t e = launch_interface_batched(b->ws + b->o_bif[k], nt, k, b->Jmax, b->if_cols[k], b->if_s[k],
                                                    b->if_cw, main);
      if (e != hipSuccess) {
        restore();
        return tt_fail(TT_ERR_HIP, "interface launch failed: %s", hipGetErrorString(e));
      }
    }
    TT_HIP_TRY(hipStreamWaitEvent(main, b->ev_step[k], 0));
    const BUpd* du = reinterpret_cast<const BUpd*>(b->ws + b->o_upd[k]);
    TT_HIP_TRY(launch_gram_batched(du, nt, b->g_gx[k], main));
    TT_HIP_TRY(launch_solve_batched(du, nt, 0, b->g_count[k], b->g_cbb[k], b->g_lchol[k], b->g_ltrsm[k], main));
    const int32_t* dq = reinterpret_cast<const int32_t*>(b->ws + b->o_qidx[k]);
    for (const auto& c : b->qcls[k]) TT_HIP_TRY(launch_qr_batched(du, dq + c.off, c.cnt, c.rmax, c.rpt, main));
    for (int32_t i : b->qfall[k]) {
      tt_plan p = b->plans[i];
      p->stream = main;
      double* const* G = reinterpret_cast<double* const*>(cores[i]);
      const int64_t m = p->r[k] * p->n[k], r = p->r[k + 1];
      TT_HIP_TRY(launch_qr_core(p, G[k], m, r, 1, m));
      TT_HIP_TRY(launch_absorb_left(p, G[k + 1], r, p->n[k + 1] * p->r[k + 2]));
      p->stream = keep[i];
    }
    // R of the batched QRs into core k + 1 (the per-problem QRs above absorbed
    // theirs; their descriptors carry no next core)
    TT_HIP_TRY(launch_absorb_left_batched(du, nt, b->g_cols[k], main));
  }
  // next sweep's tables, once the sketches (side stream) and the interface
  // sketches (batch stream) have read the current ones
  if (tables_batched) {
    TT_HIP_TRY(hipStreamWaitEvent(main, b->ev_done, 0));
    for (tt_plan p : b->plans) p->sweep += 1;
    TT_HIP_TRY(launch_gen_tables_batched(b->ws + b->o_tabargs, b->count, b->tab_max, main));
    return TT_OK;
  }
  TT_HIP_TRY(hipEventRecord(b->ev_main, main));
  for (int l = 0; l < kLanes; ++l) TT_HIP_TRY(hipStreamWaitEvent(b->lane[l], b->ev_main, 0));
  for (int i = 0; i < b->count; ++i) {
    tt_plan p = b->plans[i];
    p->stream = lane_of(i);
    const hipError_t e = hipStreamWaitEvent(p->stream, b->ev_done, 0);
    if (e != hipSuccess || (st = tt_sweep_end(p))) {
      restore();
      return e != hipSuccess ? tt_fail(TT_ERR_HIP, "hipStreamWaitEvent failed") : st;
    }
  }
  restore();
  for (int l = 0; l < kLanes; ++l) {
    TT_HIP_TRY(hipEventRecord(b->ev_lane[l], b->lane[l]));
    TT_HIP_TRY(hipStreamWaitEvent(main, b->ev_lane[l], 0));
  }
  TT_HIP_TRY(hipStreamWaitEvent(main, b->ev_done, 0));
  return TT_OK;
}

void drop_graph(tt_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->cap_ptrs.clear();
}

}  // namespace

namespace {

// average milliseconds of `reps` calls of f after one warm call
template <typename F>
tt_status time_ms(tt_batch b, hipEvent_t e0, hipEvent_t e1, int reps, F f, float* ms) {
  TT_HIP_TRY(f());
  TT_HIP_TRY(hipEventRecord(e0, b->stream));
  for (int r = 0; r < reps; ++r) TT_HIP_TRY(f());
  TT_HIP_TRY(hipEventRecord(e1, b->stream));
  TT_HIP_TRY(hipEventSynchronize(e1));
  TT_HIP_TRY(hipEventElapsedTime(ms, e0, e1));
  *ms /= (float)reps;
  return TT_OK;
}

bool nj_ok(tt_batch b, int nj) { return nj == 4 || (nj == 2 && b->max_n0 <= 128); }

// fibres (or, on slab steps, 64-entry rows) per lane group in flight
std::vector<int> fib_choices(tt_batch b, int k) {
  if (k == 0) return {4, 8};
  if (b->slab[k]) return b->ssort[k] ? std::vector<int>{1, 2, 4, 8} : std::vector<int>{4, 8};
  return {8, 16};
}

tt_status autotune_body(tt_batch b, int reps, hipEvent_t e0, hipEvent_t e1) {
  tt_status st;
  float ms = 0.0f;
  for (int k = 0; k < b->max_d; ++k) {
    if (b->tids[k].empty()) continue;
    // data sketch of step k
    float best = 1e30f;
    int bnj = b->nj[k], bfib = b->fib[k];
    int64_t bW = b->W[k];
    for (int nj : {2, 4}) {
      if (!nj_ok(b, nj)) continue;
      for (int fib : fib_choices(b, k)) {
        if (b->slab[k] && nj != b->nj[k]) continue;   // the slab kernel reads whole rows
        b->nj[k] = nj;
        b->fib[k] = fib;
        std::vector<int64_t> cand{0};
        if (k >= 1) {
          const int64_t res = occupancy_grid(b, k, nj, fib);
          cand = {res / 2, res, 2 * res, 4 * res, 8 * res};
        }
        for (int64_t W : cand) {
          if (k >= 1 && (W < 1 || W > b->Wmax)) continue;
          if ((st = time_ms(b, e0, e1, reps, [&]() { return launch_step_sketch(b, k, W); }, &ms))) return st;
          if (ms < best) {
            best = ms;
            bnj = nj;
            bfib = fib;
            bW = W;
          }
        }
      }
    }
    b->nj[k] = bnj;
    b->fib[k] = bfib;
    b->W[k] = bW;
    // Gram K-chunk of step k's core updates (contents of SH and Y do not
    // matter for the timing; the Cholesky is not run)
    const int32_t nt = (int32_t)b->upd[k].size();
    float gbest = 1e30f;
    int32_t bkc = b->kchunk[k];
    for (int32_t kc : {256, 512, 1024}) {
      set_kchunk(b, k, kc);
      TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_upd[k], b->upd[k].data(), sizeof(BUpd) * nt, hipMemcpyHostToDevice,
                                b->stream));
      const BUpd* du = reinterpret_cast<const BUpd*>(b->ws + b->o_upd[k]);
      auto gram = [&]() -> hipError_t {
        const hipError_t e = launch_gram_batched(du, nt, b->g_gx[k], b->stream);
        return e != hipSuccess ? e : launch_gram_sum_batched(du, nt, b->g_count[k], b->stream);
      };
      if ((st = time_ms(b, e0, e1, reps, gram, &ms))) return st;
      if (ms < gbest) {
        gbest = ms;
        bkc = kc;
      }
    }
    set_kchunk(b, k, bkc);
  }
  return TT_OK;
}

}  // namespace

extern "C" {

tt_status tt_batch_plan(int32_t count, const tt_plan_desc* descs, void* hip_stream, size_t* workspace_bytes,
                        tt_batch* out) {
  if (!descs || !workspace_bytes || !out) return tt_fail(TT_ERR_ARG, "null argument");
  if (count < 1 || count > TT_BATCH_MAX) return tt_fail(TT_ERR_ARG, "count=%d outside [1, %d]", count, TT_BATCH_MAX);
  tt_batch b = new (std::nothrow) tt_batch_s();
  if (!b) return tt_fail(TT_ERR_ARG, "out of host memory");
  b->count = count;
  b->stream = static_cast<hipStream_t>(hip_stream);
  size_t o = 0;
  int max_n0 = 1;
  for (int i = 0; i < count; ++i) {
    const tt_plan_desc& ds = descs[i];
    if (ds.x_dtype != TT_F32 || ds.work_dtype != TT_F32 || ds.gram_mode != TT_GRAM_WORK) {
      tt_batch_destroy(b);
      return tt_fail(TT_ERR_ARG, "problem %d: the batched form takes FP32 X and FP32 work", i);
    }
    if (ds.d < 2 || !ds.n || ds.n[0] > 256) {
      tt_batch_destroy(b);
      return tt_fail(TT_ERR_SHAPE, "problem %d: the batched form needs d >= 2 and n_0 <= 256", i);
    }
    tt_plan_desc sd = ds;
    sd.flags |= TT_FLAG_SERIAL | TT_FLAG_NO_INNER;   // the batch forms every Y_k itself
    size_t ws = 0;
    tt_plan p = nullptr;
    const tt_status st = tt_sketch_plan(&sd, hip_stream, &ws, &p);
    if (st) {
      tt_batch_destroy(b);
      return st;
    }
    b->plans.push_back(p);
    if (p->N / p->n[0] > (int64_t)UINT32_MAX) {   // fibre indices are 32-bit in the batched sketch
      tt_batch_destroy(b);
      return tt_fail(TT_ERR_SHAPE, "problem %d: more than 2^32 mode-0 fibres for the batched form", i);
    }
    b->plan_off.push_back(o);
    o = align256(o + ws);
    if (p->d > b->max_d) b->max_d = p->d;
    if (p->J > b->Jmax) b->Jmax = (int32_t)p->J;
    if (p->n[0] > max_n0) max_n0 = (int)p->n[0];
  }
  // entries of a fibre per lane: at least 2, so that a lane group serves
  // two or more short fibres per load round and the per-fibre work (key and
  // offset shuffles, bucket arithmetic) is shared by more entries (measured
  // on 256 uneven TTs with n_0 in [20, 60]: 1 / 2 / 4 entries per lane gave
  // 81.7 / 73.0 / 81.1 ms per sweep)
  b->max_n0 = max_n0;
  for (int k = 0; k < TT_MAX_ORDER; ++k) {
    b->nj[k] = max_n0 <= 128 ? 2 : 4;
    b->fib[k] = k == 0 ? 8 : 16;   // slab steps: rows in flight, set below
    b->kchunk[k] = 256;
  }
  // per-step work lists: problems of order > k, their fibre and column prefixes,
  // and partial slots per column for the largest grid
  b->tids.resize(b->max_d);
  b->stids.resize(b->max_d);
  b->fpre.resize(b->max_d);
  b->cpre.resize(b->max_d);
  b->spre.resize(b->max_d);
  size_t part_max = 1;
  for (int k = 0; k < b->max_d; ++k) {
    b->W[k] = 0;
    b->fpre[k].push_back(0);
    b->cpre[k].push_back(0);
    // slab units for k >= 2 when the largest slab table and table set fit in
    // kSlabLds bytes of LDS beside the accumulator
    b->slab[k] = k >= 2;
    b->ssort[k] = k >= 2;
    for (int i = 0; i < count; ++i) {
      tt_plan p = b->plans[i];
      if (p->d <= k) continue;
      if (p->N / (p->n[0] * p->n[1]) >= ((int64_t)1 << 31)) b->ssort[k] = false;   // slab offsets carry a sign bit
      // (clamped: any value past the LDS limit only turns the slab path off)
      const int64_t S = std::min<int64_t>((int64_t)p->n[0] * p->n[1], INT32_MAX);
      const int64_t tab = std::min<int64_t>((int64_t)p->tab_off[p->d], INT32_MAX);
      b->slab_S[k] = std::max(b->slab_S[k], (int32_t)S);
      b->slab_tab[k] = std::max(b->slab_tab[k], (int32_t)tab);
    }
    if (sizeof(uint32_t) * ((size_t)b->slab_S[k] + b->slab_tab[k]) > kSlabLds) b->slab[k] = false;
    if (!b->slab[k]) b->ssort[k] = false;
    if (b->slab[k]) b->fib[k] = b->ssort[k] ? 1 : 8;   // the key-sorted slab stream by default
    for (int i = 0; i < count; ++i) {
      tt_plan p = b->plans[i];
      if (p->d <= k) continue;
      b->tids[k].push_back(i);
      if (k == 1 && tt_sketch_fused01(p)) {   // Y_1 from the outer sketch of step 0
        b->fids.push_back(i);
        b->fid_n1 = std::max(b->fid_n1, (int32_t)p->n[1]);
        continue;
      }
      b->stids[k].push_back(i);
      b->fpre[k].push_back(b->fpre[k].back() + p->N / p->n[0] / (b->slab[k] ? p->n[1] : 1));
      b->cpre[k].push_back(b->cpre[k].back() + p->n[k]);
    }
    const int64_t Ttot = b->fpre[k].back();
    b->spre[k].push_back(0);
    for (size_t j = 0; j < b->stids[k].size(); ++j) {
      tt_plan p = b->plans[b->stids[k][j]];
      const int64_t F = (p->N / p->n[0] / (b->slab[k] ? p->n[1] : 1)) / (k == 0 ? 1 : p->n[k]);
      // a column of F consecutive fibres meets at most floor((F - 1) W / T) + 2 ranges
      const int64_t slots = (int64_t)(((__int128)(F - 1) * b->Wmax) / (Ttot > 0 ? Ttot : 1)) + 2;
      for (int64_t c = 0; c < p->n[k]; ++c) b->spre[k].push_back(b->spre[k].back() + slots);
    }
    if (k >= 1 && (size_t)b->spre[k].back() > part_max) part_max = (size_t)b->spre[k].back();
  }
  // the largest buckets first, so that the last workgroups of the outer-sketch launch are short ones
  std::stable_sort(b->fids.begin(), b->fids.end(), [&](int32_t a, int32_t c) {
    return b->plans[a]->N / b->plans[a]->J > b->plans[c]->N / b->plans[c]->J;
  });
  b->o_desc = o;
  o = align256(o + sizeof(BTensor) * count);
  // batched core updates: shapes known now, pointers filled per call
  b->upd.resize(b->max_d);
  b->bif.resize(b->max_d);
  b->qcls.resize(b->max_d);
  b->qidx.resize(b->max_d);
  b->qfall.resize(b->max_d);
  for (int k = 0; k < b->max_d; ++k) {
    const int nt = (int)b->tids[k].size();
    b->upd[k].resize(nt);
    for (int j = 0; j < nt; ++j) {
      tt_plan p = b->plans[b->tids[k][j]];
      BUpd& u = b->upd[k][j];
      u = BUpd{};
      u.J = (int32_t)p->J;
      u.s = (int32_t)(p->r[k] * p->r[k + 1]);
      u.nk = (int32_t)p->n[k];
      u.rk = (int32_t)p->r[k];
      u.rk1 = (int32_t)p->r[k + 1];
      u.kchunk = b->kchunk[k];
      u.chunks = (int32_t)((p->J + u.kchunk - 1) / u.kchunk);
      u.lambda = p->lambda;
      const size_t np = (size_t)u.s * (u.s + 1) / 2;
      int CB = 64;
      while (CB > 1 && (np + (size_t)u.s * CB) * sizeof(double) > 150 * 1024) CB >>= 1;
      u.CB = CB;
      u.ncols_next = k + 1 < p->d ? (int32_t)(p->n[k + 1] * p->r[k + 2]) : 0;
      const int tiles = ((u.s + 15) / 16) * ((u.s + u.nk + 15) / 16);
      b->g_gx[k] = std::max(b->g_gx[k], ((tiles + 3) / 4) * u.chunks);
      b->g_count[k] = std::max(b->g_count[k], u.s * (u.s + u.nk));
      b->g_cbb[k] = std::max(b->g_cbb[k], (u.nk + CB - 1) / CB);
      b->g_cols[k] = std::max(b->g_cols[k], u.ncols_next);
      b->g_lchol[k] = std::max(b->g_lchol[k], tt_chol_lds_bytes(u.s));
      b->g_ltrsm[k] = std::max(b->g_ltrsm[k], (np + (size_t)u.s * CB) * sizeof(double));
      if (k + 1 < p->d) {
        const int64_t m = (int64_t)u.rk * u.nk;
        if (m > 4 * 512 || u.rk1 > 16) {
          b->qfall[k].push_back(b->tids[k][j]);
        } else {
          const int32_t rmax = u.rk1 <= 4 ? 4 : (u.rk1 <= 8 ? 8 : (u.rk1 <= 12 ? 12 : 16));
          const int32_t rpt = m <= 512 ? 1 : (m <= 1024 ? 2 : 4);
          size_t c = 0;
          while (c < b->qcls[k].size() && !(b->qcls[k][c].rmax == rmax && b->qcls[k][c].rpt == rpt)) ++c;
          if (c == b->qcls[k].size()) b->qcls[k].push_back({rmax, rpt, 0, 0});
          b->qcls[k][c].cnt += 1;
        }
      }
    }
    // class member lists, contiguous per class
    int32_t off = 0;
    for (auto& c : b->qcls[k]) {
      c.off = off;
      off += c.cnt;
      c.cnt = 0;
    }
    b->qidx[k].assign(off, 0);
    for (int j = 0; j < nt; ++j) {
      tt_plan p = b->plans[b->tids[k][j]];
      const BUpd& u = b->upd[k][j];
      if (k + 1 >= p->d) continue;
      const int64_t m = (int64_t)u.rk * u.nk;
      if (m > 4 * 512 || u.rk1 > 16) continue;
      const int32_t rmax = u.rk1 <= 4 ? 4 : (u.rk1 <= 8 ? 8 : (u.rk1 <= 12 ? 12 : 16));
      const int32_t rpt = m <= 512 ? 1 : (m <= 1024 ? 2 : 4);
      for (auto& c : b->qcls[k])
        if (c.rmax == rmax && c.rpt == rpt) b->qidx[k][c.off + c.cnt++] = j;
    }
    b->o_upd[k] = o;
    o = align256(o + sizeof(BUpd) * (nt + 1));
    b->o_bif[k] = o;
    o = align256(o + sizeof(BIface) * (nt + 1));
    for (int j = 0; j < nt; ++j) {
      tt_plan p = b->plans[b->tids[k][j]];
      const int32_t cols = k >= 1 ? (int32_t)(p->r[k - 1] * p->r[k]) : 0;
      b->if_cols[k] = std::max(b->if_cols[k], cols);
      b->if_s[k] = std::max(b->if_s[k], (int32_t)(p->r[k] * p->r[k + 1]));
      for (int i = 0; i <= p->d; ++i)
        while (b->if_cw < p->r[i]) b->if_cw <<= 1;
    }
    b->o_qidx[k] = o;
    o = align256(o + sizeof(int32_t) * (b->qidx[k].size() + 1));
  }
  // right-to-left orthogonalisation: QR of G_s^R transposed (n_s R_{s+1} x
  // R_s) in register classes, per-problem QRs beyond them
  b->ro.resize(b->max_d);
  b->rcls.resize(b->max_d);
  b->ridx.resize(b->max_d);
  b->rids.resize(b->max_d);
  b->rfall.resize(b->max_d);
  for (int sidx = 1; sidx < b->max_d; ++sidx) {
    for (int i = 0; i < count; ++i) {
      tt_plan p = b->plans[i];
      if (p->d <= sidx) continue;
      BRo u{};
      u.m = (int32_t)(p->n[sidx] * p->r[sidx + 1]);
      u.r = (int32_t)p->r[sidx];
      u.rows = (int32_t)(p->r[sidx - 1] * p->n[sidx - 1]);
      b->ro[sidx].push_back(u);
      b->rids[sidx].push_back(i);
      b->ro_rows[sidx] = std::max(b->ro_rows[sidx], u.rows);
    }
    auto cls = [](const BRo& u, int32_t& rmax, int32_t& rpt) {
      if (u.m > 4 * 512 || u.r > 16) return false;
      rmax = u.r <= 4 ? 4 : (u.r <= 8 ? 8 : (u.r <= 12 ? 12 : 16));
      rpt = u.m <= 512 ? 1 : (u.m <= 1024 ? 2 : 4);
      return true;
    };
    for (size_t j = 0; j < b->ro[sidx].size(); ++j) {
      int32_t rmax = 0, rpt = 0;
      if (!cls(b->ro[sidx][j], rmax, rpt)) {
        b->rfall[sidx].push_back((int32_t)j);
        continue;
      }
      size_t c = 0;
      while (c < b->rcls[sidx].size() && !(b->rcls[sidx][c].rmax == rmax && b->rcls[sidx][c].rpt == rpt)) ++c;
      if (c == b->rcls[sidx].size()) b->rcls[sidx].push_back({rmax, rpt, 0, 0});
      b->rcls[sidx][c].cnt += 1;
    }
    int32_t off = 0;
    for (auto& c : b->rcls[sidx]) {
      c.off = off;
      off += c.cnt;
      c.cnt = 0;
    }
    b->ridx[sidx].assign(off, 0);
    for (size_t j = 0; j < b->ro[sidx].size(); ++j) {
      int32_t rmax = 0, rpt = 0;
      if (!cls(b->ro[sidx][j], rmax, rpt)) continue;
      for (auto& c : b->rcls[sidx])
        if (c.rmax == rmax && c.rpt == rpt) b->ridx[sidx][c.off + c.cnt++] = (int32_t)j;
    }
    b->o_ro[sidx] = o;
    o = align256(o + sizeof(BRo) * (b->ro[sidx].size() + 1));
    b->o_ridx[sidx] = o;
    o = align256(o + sizeof(int32_t) * (b->ridx[sidx].size() + 1));
  }
  for (int i = 0; i < count; ++i) {
    tt_plan p = b->plans[i];
    int32_t cols = 0;
    for (int c = 1; c < p->d; ++c) cols += (int32_t)(p->r[c] * p->r[c + 1]);
    b->fft0_cols = std::max(b->fft0_cols, cols);
  }
  b->o_fids = o;
  o = align256(o + sizeof(int32_t) * (b->fids.size() + 1));
  b->o_zids = o;
  o = align256(o + sizeof(int32_t) * (b->fids.size() + 1));
  for (int k = 0; k < b->max_d; ++k) {
    b->o_tids[k] = o;
    o = align256(o + sizeof(int32_t) * (b->tids[k].size() + 1));
    b->o_stids[k] = o;
    o = align256(o + sizeof(int32_t) * (b->stids[k].size() + 1));
    b->o_fpre[k] = o;
    o = align256(o + sizeof(int64_t) * b->fpre[k].size());
    b->o_cpre[k] = o;
    o = align256(o + sizeof(int64_t) * b->cpre[k].size());
    b->o_spre[k] = o;
    o = align256(o + sizeof(int64_t) * b->spre[k].size());
  }
  for (int k = 0; k < b->max_d; ++k) {
    const std::vector<int32_t>& ids = k == 0 ? b->tids[0] : b->stids[k];
    b->sort_sets[k] = k == 0 || b->ssort[k] ? (int32_t)ids.size() : 0;
    b->sort_blocks[k] = 0;
    for (int32_t i = 0; i < b->sort_sets[k]; ++i) {
      tt_plan p = b->plans[ids[i]];
      b->sort_blocks[k] += (int32_t)tt_sort_chunks(k == 0 ? p->O0 : p->N / (p->n[0] * p->n[1] * p->n[k]));
    }
    b->o_sargs[k] = o;
    o = align256(o + tt_sort_args_bytes() * (b->sort_sets[k] + 1));
    b->o_ssrc[k] = o;
    o = align256(o + sizeof(int2) * (b->sort_blocks[k] + 1));
  }
  b->o_part = o;
  o = align256(o + sizeof(double) * part_max * b->Jmax);
  b->o_counter = o;
  o = align256(o + sizeof(int64_t));
  b->o_tabargs = o;
  o = align256(o + tt_tab_args_bytes() * (count + 1));
  for (int i = 0; i < count; ++i) b->tab_max = std::max(b->tab_max, (int64_t)b->plans[i]->tab_off[b->plans[i]->d]);
  b->ws_need = o;
  b->host_desc.resize(count);
  *workspace_bytes = o;
  *out = b;
  return TT_OK;
}

tt_status tt_batch_bind_workspace(tt_batch b, void* dev_ws, size_t bytes) {
  if (!b || !dev_ws) return tt_fail(TT_ERR_ARG, "null argument");
  if (bytes < b->ws_need) return tt_fail(TT_ERR_WORKSPACE, "workspace %zu bytes < required %zu", bytes, b->ws_need);
  if (((uintptr_t)dev_ws & 255) != 0) return tt_fail(TT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  b->ws = static_cast<char*>(dev_ws);
  int64_t* counter = reinterpret_cast<int64_t*>(b->ws + b->o_counter);
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, b->stream, counter, (int64_t)0);
  TT_HIP_TRY(hipGetLastError());
  for (int i = 0; i < b->count; ++i) {
    tt_plan p = b->plans[i];
    p->dsweep = counter;
    const tt_status st = tt_plan_bind_workspace(p, b->ws + b->plan_off[i], p->ws_need);
    if (st) return st;
  }
  {
    std::vector<char> targs(tt_tab_args_bytes() * (b->count + 1));
    for (int i = 0; i < b->count; ++i)
      if (tt_tab_args(b->plans[i], targs.data() + tt_tab_args_bytes() * i) != hipSuccess)
        return tt_fail(TT_ERR_STATE, "problem %d: no device sweep counter", i);
    TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_tabargs, targs.data(), tt_tab_args_bytes() * b->count,
                              hipMemcpyHostToDevice, b->stream));
    TT_HIP_TRY(hipStreamSynchronize(b->stream));
  }
  for (int k = 0; k < b->max_d; ++k) {
    if (!b->stids[k].empty())
      TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_stids[k], b->stids[k].data(), sizeof(int32_t) * b->stids[k].size(),
                                hipMemcpyHostToDevice, b->stream));
    TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_tids[k], b->tids[k].data(), sizeof(int32_t) * b->tids[k].size(),
                              hipMemcpyHostToDevice, b->stream));
    TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_fpre[k], b->fpre[k].data(), sizeof(int64_t) * b->fpre[k].size(),
                              hipMemcpyHostToDevice, b->stream));
    TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_cpre[k], b->cpre[k].data(), sizeof(int64_t) * b->cpre[k].size(),
                              hipMemcpyHostToDevice, b->stream));
    TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_spre[k], b->spre[k].data(), sizeof(int64_t) * b->spre[k].size(),
                              hipMemcpyHostToDevice, b->stream));
  }
  if (!b->fids.empty())
    TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_fids, b->fids.data(), sizeof(int32_t) * b->fids.size(),
                              hipMemcpyHostToDevice, b->stream));
  for (int k = 0; k < b->max_d; ++k)
    if (!b->qidx[k].empty())
      TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_qidx[k], b->qidx[k].data(), sizeof(int32_t) * b->qidx[k].size(),
                                hipMemcpyHostToDevice, b->stream));
  for (int k = 1; k < b->max_d; ++k)
    if (!b->ridx[k].empty())
      TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_ridx[k], b->ridx[k].data(), sizeof(int32_t) * b->ridx[k].size(),
                                hipMemcpyHostToDevice, b->stream));
  // argument sets of each step's key sorts (pointers into the plans' workspaces)
  for (int k = 0; k < b->max_d; ++k) {
    if (b->sort_sets[k] == 0) continue;
    const std::vector<int32_t>& ids = k == 0 ? b->tids[0] : b->stids[k];
    std::vector<char> sargs(tt_sort_args_bytes() * (b->sort_sets[k] + 1));
    std::vector<int2> ssrc;
    for (int32_t i = 0; i < b->sort_sets[k]; ++i) {
      int32_t nb = 0;
      char* at = sargs.data() + tt_sort_args_bytes() * i;
      const hipError_t e = k == 0 ? tt_sort_args_outer(b->plans[ids[i]], at, &nb)
                                  : tt_sort_args_slabs(b->plans[ids[i]], k, at, &nb);
      if (e != hipSuccess) return tt_fail(TT_ERR_SHAPE, "problem %d: step-%d tuples do not fit the sort", ids[i], k);
      for (int32_t w = 0; w < nb; ++w) ssrc.push_back(make_int2(i, w));
    }
    if ((int32_t)ssrc.size() != b->sort_blocks[k]) return tt_fail(TT_ERR_STATE, "sort chunks changed");
    TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_sargs[k], sargs.data(), tt_sort_args_bytes() * b->sort_sets[k],
                              hipMemcpyHostToDevice, b->stream));
    TT_HIP_TRY(hipMemcpyAsync(b->ws + b->o_ssrc[k], ssrc.data(), sizeof(int2) * ssrc.size(), hipMemcpyHostToDevice,
                              b->stream));
    TT_HIP_TRY(hipStreamSynchronize(b->stream));   // before the host arrays go out of scope
  }
  fill_upd_buffers(b);
  b->desc_valid = false;
  b->upd_key.clear();
  drop_graph(b);
  return TT_OK;
}

tt_status tt_batch_get_plan(tt_batch b, int32_t i, tt_plan* plan) {
  if (!b || !plan) return tt_fail(TT_ERR_ARG, "null argument");
  if (i < 0 || i >= b->count) return tt_fail(TT_ERR_ARG, "problem %d out of range", i);
  *plan = b->plans[i];
  return TT_OK;
}

tt_status tt_batch_set_graph(tt_batch b, int32_t enable) {
  if (!b) return tt_fail(TT_ERR_ARG, "null batch");
  drop_graph(b);
  b->use_graph = enable != 0;
  return TT_OK;
}

tt_status tt_batch_sketch_tensor(tt_batch b, const void* const* X, int32_t k, void* const* Y) {
  if (!b || !X) return tt_fail(TT_ERR_ARG, "null argument");
  if (!b->ws) return tt_fail(TT_ERR_WORKSPACE, "no workspace bound");
  if (k < 0 || k >= b->max_d) return tt_fail(TT_ERR_ARG, "k=%d out of range", k);
  for (int i = 0; i < b->count; ++i)
    if (!X[i]) return tt_fail(TT_ERR_ARG, "problem %d: null X", i);
  tt_status st;
  if ((st = upload_desc(b, X))) return st;
  // Y_1 of the problems that take it from the outer sketch needs step 0 first;
  // without Y (timing) only the launches of step k run
  if (Y && k == 1 && !b->fids.empty()) TT_HIP_TRY(launch_step_sketch(b, 0, b->W[0]));
  TT_HIP_TRY(launch_step_sketch(b, k, b->W[k]));
  if (!Y) return TT_OK;
  for (int32_t i : b->tids[k]) {
    tt_plan p = b->plans[i];
    if (!Y[i]) return tt_fail(TT_ERR_ARG, "problem %d: null Y", i);
    TT_HIP_TRY(hipMemcpyAsync(Y[i], p->at<float>(p->o_Yall) + p->J * p->tab_off[k], sizeof(float) * p->J * p->n[k],
                              hipMemcpyDeviceToDevice, b->stream));
  }
  return TT_OK;
}

tt_status tt_batch_sweep(tt_batch b, const void* const* X, void* const* const* cores, double* residuals) {
  if (!b) return tt_fail(TT_ERR_ARG, "null batch");
  if (!b->ws) return tt_fail(TT_ERR_WORKSPACE, "no workspace bound");
  tt_status st;
  if ((st = check_inputs(b, X, cores))) return st;
  if ((st = upload_desc(b, X))) return st;
  if ((st = make_lanes(b))) return st;   // streams and events exist before any capture
  if ((st = upload_upd(b, cores))) return st;
  if (!b->use_graph) {
    if ((st = enqueue_sweep(b, cores))) return st;
  } else {
    const std::vector<const void*> key = pointer_key(b, X, cores);
    if (!b->exec || key != b->cap_ptrs) {
      drop_graph(b);
      // the caller's stream may be the legacy default stream, which cannot be
      // captured: capture on a private stream, replay on the caller's
      if (!b->cap) TT_HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
      // the capture must not start before work already queued for these buffers
      TT_HIP_TRY(hipStreamSynchronize(b->stream));
      const hipStream_t user = b->stream;
      b->stream = b->cap;
      for (tt_plan p : b->plans) p->stream = p->user_stream = b->cap;
      hipGraph_t graph = nullptr;
      hipError_t ce = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
      if (ce == hipSuccess) {
        st = enqueue_sweep(b, cores);
        ce = hipStreamEndCapture(b->cap, &graph);
      }
      b->stream = user;
      for (tt_plan p : b->plans) p->stream = p->user_stream = user;
      if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      if (ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return tt_fail(TT_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ce));
      }
      // capture enqueued nothing: the host sweep indices advanced once too many
      for (int i = 0; i < b->count; ++i) b->plans[i]->sweep -= 1;
      const hipError_t ie = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        b->exec = nullptr;
        return tt_fail(TT_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
      }
      b->cap_ptrs = key;
    }
    TT_HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    for (int i = 0; i < b->count; ++i) b->plans[i]->sweep += 1;
    b->replays += 1;
  }
  if (residuals) {
    for (int i = 0; i < b->count; ++i) {
      if ((st = tt_residual(b->plans[i], X[i], cores[i], &residuals[i]))) return st;
      if ((st = tt_plan_sync_status(b->plans[i]))) return st;
    }
  }
  return TT_OK;
}

tt_status tt_batch_sketch_path(tt_batch b, int32_t k, int32_t* path) {
  if (!b || !path) return tt_fail(TT_ERR_ARG, "null argument");
  if (k < 0 || k >= b->max_d) return tt_fail(TT_ERR_ARG, "step %d outside [0, %d)", k, b->max_d);
  *path = k == 0                                    ? TT_BSKETCH_PATH_BUCKET
          : b->slab[k] && slab_sorted(b->fib[k])    ? TT_BSKETCH_PATH_SLABS_SORTED
          : b->slab[k]                              ? TT_BSKETCH_PATH_SLABS
                                                    : TT_BSKETCH_PATH_FIBRES;
  return TT_OK;
}

tt_status tt_batch_autotune(tt_batch b, const void* const* X, int32_t reps, int64_t* chosen) {
  if (!b || !X) return tt_fail(TT_ERR_ARG, "null argument");
  if (!b->ws) return tt_fail(TT_ERR_WORKSPACE, "no workspace bound");
  if (reps < 1) reps = 1;
  tt_status st;
  if ((st = upload_desc(b, X))) return st;
  hipEvent_t e0, e1;
  TT_HIP_TRY(hipEventCreate(&e0));
  TT_HIP_TRY(hipEventCreate(&e1));
  st = autotune_body(b, reps, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->upd_key.clear();   // the timing uploads carried no core pointers
  drop_graph(b);
  if (st) return st;
  if (chosen)
    for (int k = 0; k < b->max_d; ++k) chosen[k] = b->W[k];
  return TT_OK;
}

tt_status tt_batch_get_tuning(tt_batch b, int64_t* out) {
  if (!b || !out) return tt_fail(TT_ERR_ARG, "null argument");
  for (int k = 0; k < TT_MAX_ORDER; ++k) {
    int64_t* o = out + (size_t)k * TT_BATCH_TUNE_FIELDS;
    o[0] = b->W[k];
    o[1] = b->nj[k];
    o[2] = b->fib[k];
    o[3] = b->kchunk[k];
  }
  return TT_OK;
}

tt_status tt_batch_set_tuning(tt_batch b, const int64_t* in) {
  if (!b || !in) return tt_fail(TT_ERR_ARG, "null argument");
  for (int k = 0; k < b->max_d; ++k) {
    const int64_t* v = in + (size_t)k * TT_BATCH_TUNE_FIELDS;
    if (v[0] < 0 || v[0] > b->Wmax || (k == 0 && v[0] != 0))
      return tt_fail(TT_ERR_ARG, "step %d: workgroups %lld outside [0, %lld] (0 for step 0)", k, (long long)v[0],
                     (long long)b->Wmax);
    if ((v[1] != 2 && v[1] != 4) || !nj_ok(b, (int)v[1]))
      return tt_fail(TT_ERR_ARG, "step %d: entries per lane %lld (2 needs n_0 <= 128, else 4)", k, (long long)v[1]);
    const std::vector<int> fc = fib_choices(b, k);
    if (std::find(fc.begin(), fc.end(), (int)v[2]) == fc.end() || v[2] != (int)v[2])
      return tt_fail(TT_ERR_ARG, "step %d: fibres (rows, slabs) in flight %lld not among the step's choices", k,
                     (long long)v[2]);
    if (v[3] < tt_gram_chunk_min() || v[3] > 8192 || v[3] % tt_gram_chunk_min() != 0)
      return tt_fail(TT_ERR_ARG, "step %d: Gram K-chunk %lld not a multiple of %d in [%d, 8192]", k, (long long)v[3],
                     tt_gram_chunk_min(), tt_gram_chunk_min());
  }
  for (int k = 0; k < b->max_d; ++k) {
    const int64_t* v = in + (size_t)k * TT_BATCH_TUNE_FIELDS;
    b->W[k] = v[0];
    b->nj[k] = (int)v[1];
    b->fib[k] = (int)v[2];
    set_kchunk(b, k, (int32_t)v[3]);
  }
  drop_graph(b);
  return TT_OK;
}

tt_status tt_batch_destroy(tt_batch b) {
  if (!b) return TT_OK;
  drop_graph(b);
  if (b->side) {
    (void)hipStreamSynchronize(b->side);
    (void)hipStreamDestroy(b->side);
    for (int l = 0; l < kLanes; ++l) {
      (void)hipStreamSynchronize(b->lane[l]);
      (void)hipStreamDestroy(b->lane[l]);
      (void)hipEventDestroy(b->ev_lane[l]);
    }
    (void)hipEventDestroy(b->ev_fork);
    (void)hipEventDestroy(b->ev_done);
    (void)hipEventDestroy(b->ev_main);
    for (int k = 0; k < TT_MAX_ORDER; ++k) (void)hipEventDestroy(b->ev_step[k]);
  }
  if (b->cap) {
    (void)hipStreamSynchronize(b->cap);
    (void)hipStreamDestroy(b->cap);
  }
  for (tt_plan p : b->plans) tt_plan_destroy(p);
  delete b;
  return TT_OK;
}

}  // extern "C"
