// Data sketch Y_k = S_{-k} A_(k)^T (Sec. 3, (lrtt_sub4); TensorSketch of
// Sec. 2.2): a sign-weighted scatter-add of every entry of X into J buckets.
//
// X is read as a sequence of mode-0 fibres (n_0 contiguous entries).  Within a
// fibre only i_0 varies, so the hash contribution of every other mode is one
// packed key per fibre.  A wave reads fibres with 16-byte vector loads: lane
// group g (LPF lanes) takes one fibre, lane v of the group the positions
// i_0 = (v + LPF j) V + e, whose packed mode-0 table entries stay in
// registers.  Short fibres therefore share a wave (64 / LPF fibres per load).
//
//  * k >= 1: persistent grid sized to the device occupancy.  The fibres of
//    all columns i_k, column by column, are split into equal contiguous
//    ranges, one per workgroup.  A workgroup accumulates the part of its range
//    that lies in one column into a J-entry FP64 LDS array (LDS atomics),
//    writes the array as one partial of that column, and moves on to the
//    next column of its range.  A second kernel sums the partials of each
//    column in FP64 in a fixed order.  The accumulators are FP64 for every
//    work type: on gfx950 the LDS FP64 atomic add sustains about nine times
//    the rate of the FP32 one, and it makes the per-bucket sums exact to
//    FP32 rounding of the inputs.  Fibre keys are fetched 64 at a time (one
//    vector load per lane) and handed to the lane groups by shuffles.
//  * k >= 1 when a column holds at least two fibres per key (the usual case
//    for large tensors): the fibres of one column, listed once per sweep and
//    mode in order of their key c over the modes other than 0 and k (a
//    counting sort that does not depend on the column), are summed in
//    registers while the key stays the same, and only the sums are scattered
//    into the LDS buckets (h_0(i_0) + c) mod J.  This divides the LDS atomics
//    by the number of fibres per key (about N / (n_0 n_k J)).  A workgroup owns
//    one column and an equal share of the sorted list; a key split between
//    shares is completed when the partials are summed.
//  * k = 0: a fibre has one bucket (its entries differ only in i_0, the
//    unsketched mode), so one workgroup owns one bucket b and gathers the
//    fibres hashed to b: for each i_1 it visits the outer tuples (modes
//    2..d-1) whose partial hash is (b - h_1(i_1)) mod J, found in a
//    bucket-sorted list.  Accumulation is in registers; no atomics.
//  * k = 0 and k = 1 from one pass (fused): the TensorSketch of X over modes
//    2..d-1 alone, the outer sketch (a J x n_0 x n_1 tensor: row (i_1, c)
//    sums, with their signs, the fibres X(:, i_1, o) of the outer tuples o of
//    key c), is formed from X once, slab by slab: the n_0 x n_1 slabs
//    X(:, :, o) of one key are added whole.  Y_0 row b then sums rows
//    (i_1, b - h_1(i_1)) of it with the signs of i_1, and Y_1 column i_1 adds
//    row (i_1, c) value i_0 with the sign of i_0 to bucket (c + h_0(i_0)) mod
//    J.  This replaces the k = 1 pass over X by a write and two reads of
//    J n_0 n_1 values, which pays when J n_0 n_1 is small against N.
#include <type_traits>

#include "tt_internal.h"

// threads per workgroup of the k >= 1 sketch kernels
#ifndef TT_SKETCH_THREADS
#define TT_SKETCH_THREADS 256
#endif
// a k >= 1 sketch takes the key-grouped path when a column holds at least
// this many fibres per key
#ifndef TT_SKETCH_GS_MIN
#define TT_SKETCH_GS_MIN 2
#endif

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

// (+-x) as FP64 with the sign applied as a bit flip: s is 0 or 0x80000000.
__device__ __forceinline__ double signed_f64(float x, uint32_t s) { return (double)__uint_as_float(__float_as_uint(x) ^ s); }
__device__ __forceinline__ double signed_f64(uint16_t x, uint32_t s) { return (double)__uint_as_float(((uint32_t)x << 16) ^ s); }
__device__ __forceinline__ double signed_f64(double x, uint32_t s) {
  return __longlong_as_double(__double_as_longlong(x) ^ ((long long)s << 32));
}

// Bucket offsets are kept pre-scaled to LDS byte offsets (8 b): the sum of two
// offsets below 8 J wraps with one subtraction and an unsigned min.
__device__ __forceinline__ uint32_t wrap8(uint32_t b8, uint32_t J8) {
  const uint32_t t = b8 - J8;
  return t < b8 ? t : b8;
}

// V consecutive elements of X as one load (16 bytes when V * sizeof(XT) == 16)
template <typename XT, int V>
struct Vec {
  XT e[V];
};
// X is streamed once per pass: nontemporal loads keep it from displacing the
// small tables and partials in the caches.
template <typename XT, int V>
__device__ __forceinline__ Vec<XT, V> load_vec(const XT* p) {
  if constexpr (V == 1) {
    return Vec<XT, 1>{{__builtin_nontemporal_load(p)}};
  } else {
    typedef XT raw_t __attribute__((ext_vector_type(V)));
    const raw_t r = __builtin_nontemporal_load(reinterpret_cast<const raw_t*>(p));
    Vec<XT, V> out;
#pragma unroll
    for (int e = 0; e < V; ++e) out.e[e] = r[e];
    return out;
  }
}

__device__ __forceinline__ int64_t shfl64(int64_t x, int src) {
  const int lo = __shfl((int)(uint32_t)(uint64_t)x, src, 64);
  const int hi = __shfl((int)(uint32_t)((uint64_t)x >> 32), src, 64);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// workgroup that owns global fibre g when Ftot fibres are split into W ranges
__device__ __forceinline__ int64_t owner(int64_t g, int64_t W, int64_t Ftot) { return ((g + 1) * W - 1) / Ftot; }

// ---------------------------------------------------------------- k >= 1
template <typename XT, typename WT, int V, int NJ, int U>
__global__ __launch_bounds__(TT_SKETCH_THREADS) void k_sketch_modek(
    const XT* __restrict__ X, const uint32_t* __restrict__ tab0, const uint32_t* __restrict__ KI,
    const uint32_t* __restrict__ KO, double* __restrict__ part, int32_t n0, int32_t nk, int64_t M, int64_t F,
    uint32_t J, int32_t lpf_log2, int32_t maxslots) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  const int LPF = 1 << lpf_log2;
  const int G = 64 >> lpf_log2;          // fibres per load instruction
  const int g = lane >> lpf_log2;
  const int v = lane & (LPF - 1);
  // mode-0 part of the key for this lane's positions: LDS byte offset 8 h_0
  // and sign mask
  uint32_t tb[NJ][V], ts[NJ][V];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int i0 = (v + LPF * j) * V + e;
      const uint32_t t = i0 < n0 ? tab0[i0] : 0u;
      tb[j][e] = (t & TT_KEY_MASK) << 3;
      ts[j][e] = t & TT_KEY_SIGN;
    }
  const uint32_t J8 = J << 3;
  char* accb = reinterpret_cast<char*>(acc);
  const int64_t W = gridDim.x;
  const int64_t w = blockIdx.x;
  const int64_t Ftot = (int64_t)nk * F;
  const int64_t gs = w * Ftot / W, ge = (w + 1) * Ftot / W;
  for (int64_t c = gs / F; gs < ge && c * F < ge; ++c) {
    const int64_t qa = (gs > c * F ? gs : c * F) - c * F;
    const int64_t qe = (ge < (c + 1) * F ? ge : (c + 1) * F) - c * F;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) acc[b] = 0.0;
    __syncthreads();
    const int64_t wa = qa + (qe - qa) * wv / NW, we = qa + (qe - qa) * (wv + 1) / NW;
    for (int64_t qb = wa; qb < we; qb += 64) {
      // keys and element offsets of the next (up to) 64 fibres, one per lane
      const int64_t ql = qb + lane;
      uint32_t keyl = 0;
      int64_t offl = 0;
      if (ql < we) {
        const int64_t rho = ql / M, mu = ql - rho * M;
        keyl = key_add(KI[mu], KO[rho], J);
        offl = ((rho * nk + c) * M + mu) * (int64_t)n0;
      }
      const uint32_t kbl = (keyl & TT_KEY_MASK) << 3, ksl = keyl & TT_KEY_SIGN;
      const int nb = (we - qb) < 64 ? (int)(we - qb) : 64;
      for (int t = 0; t < nb; t += G * U) {
        Vec<XT, V> x[U][NJ];
        uint32_t kb[U], ks[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = t + u * G + g;
          ok[u] = idx < nb;
          kb[u] = __shfl(kbl, idx & 63, 64);
          ks[u] = __shfl(ksl, idx & 63, 64);
          const int64_t off = shfl64(offl, idx & 63);
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const int p = (v + LPF * j) * V;
            if (ok[u] && p < n0) x[u][j] = load_vec<XT, V>(X + off + p);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const int p = (v + LPF * j) * V;
            if (ok[u] && p < n0) {
#pragma unroll
              for (int e = 0; e < V; ++e) {
                const uint32_t b8 = wrap8(tb[j][e] + kb[u], J8);
                atomicAdd(reinterpret_cast<double*>(accb + b8), signed_f64(x[u][j].e[e], ts[j][e] ^ ks[u]));
              }
            }
          }
      }
    }
    __syncthreads();
    const int64_t slot = w - owner(c * F, W, Ftot);
    double* out = part + ((int64_t)c * maxslots + slot) * (int64_t)J;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) out[b] = acc[b];
    __syncthreads();
  }
}

// Y[b + J c] = sum over the partials of column c, in FP64, in slot order.
template <typename WT>
__global__ void k_reduce_parts(const double* __restrict__ part, WT* __restrict__ Y, int64_t J, int64_t nk, int64_t F,
                               int64_t W, int32_t maxslots) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= J * nk) return;
  const int64_t c = idx / J, b = idx - c * J;
  const int64_t Ftot = nk * F;
  const int64_t cnt = owner((c + 1) * F - 1, W, Ftot) - owner(c * F, W, Ftot) + 1;
  const double* p = part + c * maxslots * J + b;
  double s = 0.0;
  for (int64_t q = 0; q < cnt; ++q) s += p[q * J];
  Y[idx] = (WT)s;
}

// Y_1 from the outer sketch of the fused k = 0 pass.  Workgroup (s, i_1)
// scatters rows (c, i_1) for c in [s J / S, (s + 1) J / S) (row c holds the
// outer tuples of key c; its value i_0 goes to bucket (c + h_0(i_0)) mod J)
// into a J-entry FP64 LDS array and writes it as partial s of column i_1.
// V: values per load (n_0 a multiple of V).
template <typename WT, int V>
__global__ __launch_bounds__(256) void k_sketch_y1_outer(const WT* __restrict__ zo, const uint32_t* __restrict__ tab0,
                                                         double* __restrict__ part, int32_t n0, int32_t n1, uint32_t J,
                                                         int32_t S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  uint32_t* t0 = reinterpret_cast<uint32_t*>(acc + ((J + 1) & ~1u));   // 16-byte aligned
  const int s = blockIdx.x, i1 = blockIdx.y;
  for (uint32_t q = threadIdx.x; q < J; q += blockDim.x) acc[q] = 0.0;
  for (int q = threadIdx.x; q < n0; q += blockDim.x) t0[q] = tab0[q];
  __syncthreads();
  const uint32_t r0 = (uint32_t)((int64_t)s * J / S), r1 = (uint32_t)((int64_t)(s + 1) * J / S);
  const uint32_t nv = (r1 - r0) * (uint32_t)(n0 / V);   // vectors in the range (< 2^31)
  const uint32_t vpr = (uint32_t)(n0 / V);
  const int64_t Sz = (int64_t)n0 * n1;                  // one outer key's rows
  const WT* base = zo + (int64_t)r0 * Sz + (int64_t)i1 * n0;
  for (uint32_t q = threadIdx.x; q < nv; q += blockDim.x) {
    const uint32_t r = q / vpr;
    const uint32_t i0 = (q - r * vpr) * V;
    const Vec<WT, V> x = load_vec<WT, V>(base + (int64_t)r * Sz + i0);
    const uint32_t c = r0 + r;   // the outer key of the row
    uint32_t tv[V];   // the V mode-0 entries in one LDS read (i0 is a multiple of V)
    if constexpr (V == 4) {
      const uint4 w = *reinterpret_cast<const uint4*>(t0 + i0);
      tv[0] = w.x;
      tv[1] = w.y;
      tv[2] = w.z;
      tv[3] = w.w;
    } else if constexpr (V == 2) {
      const uint2 w = *reinterpret_cast<const uint2*>(t0 + i0);
      tv[0] = w.x;
      tv[1] = w.y;
    } else {
      tv[0] = t0[i0];
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const uint32_t t = tv[e];
      uint32_t b = c + (t & TT_KEY_MASK);
      b = b >= J ? b - J : b;
      atomicAdd(&acc[b], signed_f64(x.e[e], t & TT_KEY_SIGN));
    }
  }
  __syncthreads();
  double* out = part + ((int64_t)i1 * S + s) * (int64_t)J;
  for (uint32_t q = threadIdx.x; q < J; q += blockDim.x) out[q] = acc[q];
}

// Y[b + J c] = the sum of the S partials of column c, in FP64, in slot order.
template <typename WT>
__global__ void k_reduce_slots(const double* __restrict__ part, WT* __restrict__ Y, int64_t J, int64_t nk, int32_t S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= J * nk) return;
  const int64_t c = idx / J, b = idx - c * J;
  const double* p = part + c * S * J + b;
  double acc = 0.0;
  for (int q = 0; q < S; ++q) acc += p[(int64_t)q * J];
  Y[idx] = (WT)acc;
}

// ---------------------------------------------------------------- k >= 1, key-grouped
// DB (double-buffered): the loads of the next batch of fibres are issued
// before the current batch is summed, so a wave always has loads in flight.
// It pays when one fibre fills the wave (one fibre per load, long fibres);
// for short fibres the second buffer costs more occupancy than it gains.
template <typename XT, typename WT, int V, int NJ, int U, bool DB>
__global__ __launch_bounds__(TT_SKETCH_THREADS) void k_sketch_gs(
    const XT* __restrict__ X, const uint32_t* __restrict__ tab0, const uint2* __restrict__ list,
    double* __restrict__ part, int32_t n0, int32_t nk, int64_t M, int64_t F, uint32_t J, int32_t lpf_log2,
    int32_t maxslots) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  const int LPF = 1 << lpf_log2;
  const int G = 64 >> lpf_log2;
  const int g = lane >> lpf_log2;
  const int v = lane & (LPF - 1);
  uint32_t tb[NJ][V], ts[NJ][V];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int i0 = (v + LPF * j) * V + e;
      const uint32_t t = i0 < n0 ? tab0[i0] : 0u;
      tb[j][e] = (t & TT_KEY_MASK) << 3;
      ts[j][e] = t & TT_KEY_SIGN;
    }
  const uint32_t J8 = J << 3;
  char* accb = reinterpret_cast<char*>(acc);
  // this workgroup's share of the (column, list entry) sequence
  const int64_t W = gridDim.x;
  const int64_t w = blockIdx.x;
  const int64_t Ftot = (int64_t)nk * F;
  const int64_t gs = w * Ftot / W, ge = (w + 1) * Ftot / W;
  for (int64_t c = gs / F; gs < ge && c * F < ge; ++c) {
    const int64_t qa = (gs > c * F ? gs : c * F) - c * F;
    const int64_t qe = (ge < (c + 1) * F ? ge : (c + 1) * F) - c * F;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) acc[b] = 0.0;
    __syncthreads();
    const int64_t wa = qa + (qe - qa) * wv / NW, we = qa + (qe - qa) * (wv + 1) / NW;
    const XT* Xc = X + c * M * (int64_t)n0;
    double sacc[NJ][V];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int e = 0; e < V; ++e) sacc[j][e] = 0.0;
    uint32_t cur = 0xffffffffu;   // key of the running sums (none yet)
    auto flush = [&]() {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int p = (v + LPF * j) * V;
        if (p < n0)
#pragma unroll
          for (int e = 0; e < V; ++e) {
            const uint32_t b8 = wrap8(tb[j][e] + (cur << 3), J8);
            atomicAdd(reinterpret_cast<double*>(accb + b8), signed_f64(sacc[j][e], ts[j][e]));
            sacc[j][e] = 0.0;
          }
      }
    };
    // a batch: the fibres off + u G + g of the current chunk of 64 list
    // entries, fibre u G + g to lane group g; off + u G + g stays below 64
    auto issue = [&](const uint2& itl, int off, int64_t left, uint32_t (&ix)[U], uint32_t (&iy)[U], bool (&ok)[U],
                     Vec<XT, V> (&x)[U][NJ]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = off + u * G + g;
        ok[u] = u * G < 64 && u * G + g < left;
        ix[u] = (uint32_t)__shfl((int)itl.x, idx & 63, 64);
        iy[u] = (uint32_t)__shfl((int)itl.y, idx & 63, 64);
        const XT* base = Xc + (int64_t)(ix[u] & TT_KEY_MASK) * n0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int p = (v + LPF * j) * V;
          if (ok[u] && p < n0) x[u][j] = load_vec<XT, V>(base + p);
        }
      }
    };
    auto consume = [&](const uint32_t (&ix)[U], const uint32_t (&iy)[U], const bool (&ok)[U],
                       const Vec<XT, V> (&x)[U][NJ]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ok[u]) {
          if (iy[u] != cur) {
            if (cur != 0xffffffffu) flush();
            cur = iy[u];
          }
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const int p = (v + LPF * j) * V;
            if (p < n0)
#pragma unroll
              for (int e = 0; e < V; ++e) sacc[j][e] += signed_f64(x[u][j].e[e], ix[u] & TT_KEY_SIGN);
          }
        }
      }
    };
    const int64_t n = we - wa;
    uint32_t ixa[U], iya[U];
    bool oka[U];
    Vec<XT, V> xa[U][NJ];
    // list entries are fetched 64 at a time, one per lane, one chunk ahead,
    // so that the loads of X never wait on a list load issued just before
    if constexpr (DB) {
      const int B = G * U < 64 ? G * U : 64;
      uint2 lc = lane < n ? list[wa + lane] : make_uint2(0u, 0u);
      uint2 ln = 64 + lane < n ? list[wa + 64 + lane] : make_uint2(0u, 0u);
      uint32_t ixb[U], iyb[U];
      bool okb[U];
      Vec<XT, V> xb[U][NJ];
      auto next = [&](int64_t e0) {   // the chunk of entries [e0, e0 + 64) becomes current
        if ((e0 & 63) == 0) {
          lc = ln;
          ln = e0 + 64 + lane < n ? list[wa + e0 + 64 + lane] : make_uint2(0u, 0u);
        }
      };
      if (n > 0) issue(lc, 0, n, ixa, iya, oka, xa);
      for (int64_t e0 = 0; e0 < n; e0 += 2 * B) {
        if (e0 + B < n) {
          next(e0 + B);
          issue(lc, (int)((e0 + B) & 63), n - e0 - B, ixb, iyb, okb, xb);
        }
        consume(ixa, iya, oka, xa);
        if (e0 + B >= n) break;
        if (e0 + 2 * B < n) {
          next(e0 + 2 * B);
          issue(lc, (int)((e0 + 2 * B) & 63), n - e0 - 2 * B, ixa, iya, oka, xa);
        }
        consume(ixb, iyb, okb, xb);
      }
    } else {
      uint2 nxt = lane < n ? list[wa + lane] : make_uint2(0u, 0u);
      for (int64_t eb = 0; eb < n; eb += 64) {
        const uint2 itl = nxt;
        if (eb + 64 + lane < n) nxt = list[wa + eb + 64 + lane];
        const int nb = (n - eb) < 64 ? (int)(n - eb) : 64;
        for (int t = 0; t < nb; t += G * U) {
          issue(itl, t, nb - t, ixa, iya, oka, xa);
          consume(ixa, iya, oka, xa);
        }
      }
    }
    if (cur != 0xffffffffu) flush();
    __syncthreads();
    const int64_t slot = w - owner(c * F, W, Ftot);
    double* out = part + ((int64_t)c * maxslots + slot) * (int64_t)J;
    for (uint32_t b = threadIdx.x; b < J; b += blockDim.x) out[b] = acc[b];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- k = 0
// ---------------------------------------------------------------- k = 0
template <typename XT, typename WT, int V, int NJ, int U>
__global__ __launch_bounds__(256) void k_sketch_mode0(
    const XT* __restrict__ X, const uint32_t* __restrict__ tab1, const uint32_t* __restrict__ off,
    const uint32_t* __restrict__ sorted, WT* __restrict__ Y, int32_t n0, int32_t n1, uint32_t J, int32_t i0_lo,
    int32_t i0_cnt, int32_t lpf_log2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* red = reinterpret_cast<double*>(smem_raw);   // NW x (64 * NJ * V)
  const uint32_t b = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  const int LPF = 1 << lpf_log2;
  const int G = 64 >> lpf_log2;
  const int g = lane >> lpf_log2;
  const int v = lane & (LPF - 1);
  // FP64 sums: exact enough that the order in which fibres arrive does not
  // show in the FP32 result
  double acc[NJ][V];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int e = 0; e < V; ++e) acc[j][e] = 0.0;

  // the i_1 of this wave (i_1 = wv + NW q) are taken 64 at a time: lane q
  // fetches the table entry and list segment of one of them, and the first
  // 64 list entries of the next segment are loaded before the fibres of the
  // current one, so the loads of X never wait on a list load issued just
  // before them
  for (int i1b = wv; i1b < n1; i1b += NW * 64) {
    const int i1l = i1b + NW * lane;
    uint32_t t1l = 0, begl = 0, endl = 0;
    if (i1l < n1) {
      t1l = tab1[i1l];
      const uint32_t h1 = t1l & TT_KEY_MASK;
      const uint32_t c = b >= h1 ? b - h1 : b + J - h1;
      begl = off[c];
      endl = off[c + 1];
    }
    const int nq0 = (n1 - i1b + NW - 1) / NW;
    const int nq = nq0 < 64 ? nq0 : 64;
    uint32_t nxt;
    {
      const uint32_t nb0 = (uint32_t)__shfl((int)begl, 0, 64), ne0 = (uint32_t)__shfl((int)endl, 0, 64);
      nxt = (nb0 + lane < ne0) ? sorted[nb0 + lane] : 0u;
    }
    // a batch: fibres t + u G + g of the list chunk starting at e0 of the
    // segment of i_1
    auto issue = [&](uint32_t itl, int t, int nb, uint32_t t1, int i1, Vec<XT, V> (&x)[U][NJ], uint32_t (&sg)[U],
                     bool (&ok)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = t + u * G + g;
        ok[u] = idx < nb;
        const uint32_t item = (uint32_t)__shfl((int)itl, idx & 63, 64);
        sg[u] = (item ^ t1) & TT_KEY_SIGN;
        const XT* base = X + ((int64_t)(item & TT_KEY_MASK) * n1 + i1) * (int64_t)n0 + i0_lo;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int p = (v + LPF * j) * V;
          if (ok[u] && p < i0_cnt) x[u][j] = load_vec<XT, V>(base + p);
        }
      }
    };
    auto consume = [&](const Vec<XT, V> (&x)[U][NJ], const uint32_t (&sg)[U], const bool (&ok)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int p = (v + LPF * j) * V;
          if (ok[u] && p < i0_cnt)
#pragma unroll
            for (int e = 0; e < V; ++e) acc[j][e] += signed_f64(x[u][j].e[e], sg[u]);
        }
    };
    Vec<XT, V> xa[U][NJ];
    uint32_t sga[U];
    bool oka[U];
    for (int q = 0; q < nq; ++q) {
      const uint32_t t1 = (uint32_t)__shfl((int)t1l, q, 64);
      const uint32_t beg = (uint32_t)__shfl((int)begl, q, 64), end = (uint32_t)__shfl((int)endl, q, 64);
      const int i1 = i1b + NW * q;
      const uint32_t first = nxt;
      if (q + 1 < nq) {
        const uint32_t nb1 = (uint32_t)__shfl((int)begl, q + 1, 64), ne1 = (uint32_t)__shfl((int)endl, q + 1, 64);
        nxt = (nb1 + lane < ne1) ? sorted[nb1 + lane] : 0u;
      }
      for (uint32_t e0 = beg; e0 < end; e0 += 64) {
        const uint32_t itl = e0 == beg ? first : ((e0 + lane < end) ? sorted[e0 + lane] : 0u);
        const int nb = (end - e0) < 64u ? (int)(end - e0) : 64;
        for (int t = 0; t < nb; t += G * U) {
          issue(itl, t, nb, t1, i1, xa, sga, oka);
          consume(xa, sga, oka);
        }
      }
    }
  }
  // lane groups hold partial sums of the same positions: fold them
  for (int m = LPF; m < 64; m <<= 1)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int e = 0; e < V; ++e) acc[j][e] += __shfl_xor(acc[j][e], m, 64);
  constexpr int PW = 64 * NJ * V;   // positions per wave slot
  if (g == 0)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int e = 0; e < V; ++e) red[wv * PW + (v + LPF * j) * V + e] = acc[j][e];
  __syncthreads();
  for (int i = threadIdx.x; i < i0_cnt; i += blockDim.x) {
    double s = 0.0;
    for (int ww = 0; ww < NW; ++ww) s += red[ww * PW + i];
    Y[(int64_t)b + (int64_t)J * (i0_lo + i)] = (WT)s;
  }
}

// ---------------------------------------------------------------- k = 0 and the outer sketch
// The fused k = 0 pass, slab by slab.  Workgroup (piece, c) adds its piece
// of the n_0 x n_1 slabs X(:, :, o) of the outer tuples o hashed to bucket c
// (modes 2..d-1), each with its sign, and writes the sum to the outer sketch
// zo[c n_0 n_1 + i_1 n_0 + i_0] (one contiguous piece per workgroup).  Each
// slab is contiguous and read by one
// workgroup per piece, so a 128-byte line is fetched twice only where two
// slabs or pieces meet.  Values are read as V-entry vectors (every slab
// starts on a V-entry boundary when n_0 n_1 and the address of X allow it);
// a group of TPI lanes (64, 128 or 256, the fewest that cover a piece of
// 256 MV vectors with MV per lane) sums one slab at a time in FP64 registers,
// U slabs per load batch, the 256 / TPI groups splitting the bucket's list
// and adding up in a fixed order at the end.  Y_0 and Y_1 are then formed
// from the outer sketch by the two kernels below.
template <typename XT, int V>
__device__ __forceinline__ Vec<XT, V> load_vec_plain(const XT* p) {
  // plain (L2-allocating) loads: two load instructions that share a line
  // fetch it once
  typedef const XT __attribute__((address_space(1)))* gxt;
  if constexpr (V == 1) {
    return Vec<XT, 1>{{*(gxt)p}};
  } else {
    typedef XT raw_t __attribute__((ext_vector_type(V)));
    typedef const raw_t __attribute__((address_space(1)))* graw;
    const raw_t r = *(graw)p;
    Vec<XT, V> out;
#pragma unroll
    for (int e = 0; e < V; ++e) out.e[e] = r[e];
    return out;
  }
}

template <typename XT, typename WT, int V, int MV, int U>
__global__ __launch_bounds__(256) void k_sketch_zo(const XT* __restrict__ X, const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ sorted, WT* __restrict__ zo,
                                                   int64_t S) {
  __shared__ double red[3 * 64 * MV * V];   // groups 1..3 (TPI = 64) or group 1 (TPI = 128)
  const uint32_t c = blockIdx.y;
  const int64_t Sv = S / V;
  const int tpi = Sv <= 64 * MV ? 64 : Sv <= 128 * MV ? 128 : 256;
  const int ipw = 256 / tpi;
  const int grp = threadIdx.x / tpi, li = threadIdx.x - grp * tpi;
  const int64_t p0 = (int64_t)blockIdx.x * tpi * MV;   // first vector of the piece
  if (p0 >= Sv) return;
  const int plen = (int)(Sv - p0 < (int64_t)tpi * MV ? Sv - p0 : (int64_t)tpi * MV);
  const int ms = (plen + tpi - 1) / tpi;
  const uint32_t beg = off[c], end = off[c + 1];
  double acc[MV][V];
#pragma unroll
  for (int m = 0; m < MV; ++m)
#pragma unroll
    for (int i = 0; i < V; ++i) acc[m][i] = 0.0;
  for (uint32_t e0 = beg + grp; e0 < end; e0 += ipw * U) {
    Vec<XT, V> x[U][MV];
    uint32_t sg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {   // all loads first, then the sums
      const uint32_t e = e0 + ipw * u;
      const bool ok = e < end;
      const uint32_t item = ok ? sorted[e] : 0u;
      sg[u] = item & TT_KEY_SIGN;
      const XT* base = X + (int64_t)(item & TT_KEY_MASK) * S + (p0 + li) * V;
#pragma unroll
      for (int m = 0; m < MV; ++m) {
        if (ok && m < ms && li + tpi * m < plen) {
          x[u][m] = load_vec_plain<XT, V>(base + (int64_t)tpi * m * V);
        } else {
#pragma unroll
          for (int i = 0; i < V; ++i) x[u][m].e[i] = XT(0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)   // in list order
#pragma unroll
      for (int m = 0; m < MV; ++m)
#pragma unroll
        for (int i = 0; i < V; ++i) acc[m][i] += signed_f64(x[u][m].e[i], sg[u]);
  }
  if (ipw > 1) {
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
  WT* out = zo + (int64_t)c * S;
  if (grp == 0)
#pragma unroll
    for (int m = 0; m < MV; ++m)
      if (m < ms && li + tpi * m < plen) {
        const int64_t e = (p0 + li + tpi * m) * V;   // slab position of the vector's first value
#pragma unroll
        for (int i = 0; i < V; ++i) out[e + i] = (WT)acc[m][i];
      }
}

// Y_0 from the outer sketch: row b of Y_0 adds, for every i_1, row
// ((b - h_1(i_1)) mod J, i_1) of the sketch with the sign of i_1.  Thread t
// keeps i_0 = t + 256 j (j < NJ0, n_0 <= 256 NJ0) in FP64 registers; R rows
// are loaded before they are added.
template <typename WT, int NJ0>
__global__ __launch_bounds__(256) void k_sketch_y0_zo(const WT* __restrict__ zo, const uint32_t* __restrict__ tab1,
                                                      WT* __restrict__ Y, int32_t n0, int32_t n1, uint32_t J) {
  constexpr int R = 16 / NJ0;
  typedef const WT __attribute__((address_space(1)))* gwt;
  const uint32_t b = blockIdx.x;
  double acc[NJ0];
#pragma unroll
  for (int j = 0; j < NJ0; ++j) acc[j] = 0.0;
  for (int r0 = 0; r0 < n1; r0 += R) {
    WT x[R][NJ0];
    uint32_t sg[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i1 = r0 + u;
      const bool ok = i1 < n1;
      const uint32_t t1 = ok ? tab1[i1] : 0u;
      const uint32_t h1 = t1 & TT_KEY_MASK;
      const uint32_t c = b >= h1 ? b - h1 : b + J - h1;
      sg[u] = t1 & TT_KEY_SIGN;
      const gwt row = (gwt)(zo + ((int64_t)c * n1 + i1) * n0);
#pragma unroll
      for (int j = 0; j < NJ0; ++j) {
        const int i0 = threadIdx.x + 256 * j;
        x[u][j] = ok && i0 < n0 ? row[i0] : WT(0);
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int j = 0; j < NJ0; ++j) acc[j] += signed_f64(x[u][j], sg[u]);
  }
#pragma unroll
  for (int j = 0; j < NJ0; ++j) {
    const int i0 = threadIdx.x + 256 * j;
    if (i0 < n0) Y[b + (int64_t)J * i0] = (WT)acc[j];
  }
}

// ---------------------------------------------------------------- inner sketch
// The TensorSketch of every slab X(:, ..., :, o) over modes 0..m-1 alone
// (m = 2 unless the plan groups more modes): row o of Z holds, at bucket
// (h_0(i_0) + ... + h_{m-1}(i_{m-1})) mod J, the sum of
// v_0(i_0) ... v_{m-1}(i_{m-1}) X(i_0, ..., i_{m-1}, o).  Workgroup o reads
// its slab once, row by row (a row: n_0 values at fixed i_1..i_{m-1}, whose
// packed key over modes 1..m-1 is rkey[row]; the lane layout of the fibre
// kernels: LPF lanes per row, the lane's mode-0 table entries in registers,
// U rows per wave in flight), adds every entry into J FP64 LDS buckets, and
// writes them as row o of Z.  Y_k for k >= m then follows from Z
// (k_sketch_y_zi) without a pass over X of its own.
template <typename XT, typename WT, int V, int NJ, int U>
__global__ __launch_bounds__(256) void k_sketch_zi(const XT* __restrict__ X, const uint32_t* __restrict__ tab0,
                                                   const uint32_t* __restrict__ rkey, WT* __restrict__ Z, int32_t n0,
                                                   int32_t n1, uint32_t J, int lpf_log2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  uint32_t* t1 = reinterpret_cast<uint32_t*>(acc + J);
  const int64_t o = blockIdx.x;
  for (uint32_t q = threadIdx.x; q < J; q += 256) acc[q] = 0.0;
  for (int q = threadIdx.x; q < n1; q += 256) t1[q] = rkey[q];   // n1: rows of a slab
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lpf = 1 << lpf_log2, g = lane >> lpf_log2, v = lane & (lpf - 1);
  const int rw = 64 >> lpf_log2;   // rows per wave and load
  uint32_t k0[NJ][V];
  bool in0[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int i0 = (v + lpf * j) * V;
    in0[j] = i0 < n0;   // n_0 is a multiple of V: the whole vector is in range
#pragma unroll
    for (int e = 0; e < V; ++e) k0[j][e] = in0[j] ? tab0[i0 + e] : 0u;
  }
  __syncthreads();
  const XT* slab = X + o * (int64_t)n0 * n1;
  for (int r0 = wave * U * rw; r0 < n1; r0 += 4 * U * rw) {
    Vec<XT, V> x[U][NJ];
#pragma unroll
    for (int u = 0; u < U; ++u) {   // all loads first, then the sums
      const int r = r0 + u * rw + g;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if (r < n1 && in0[j]) {
          x[u][j] = load_vec_plain<XT, V>(slab + (int64_t)r * n0 + (v + lpf * j) * V);
        } else {
#pragma unroll
          for (int e = 0; e < V; ++e) x[u][j].e[e] = XT(0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + u * rw + g;
      if (r >= n1) continue;
      const uint32_t K = t1[r];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if (!in0[j]) continue;
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const uint32_t b = key_add(k0[j][e], K, J);
          atomicAdd(&acc[b & TT_KEY_MASK], signed_f64(x[u][j].e[e], b & TT_KEY_SIGN));
        }
      }
    }
  }
  __syncthreads();
  WT* out = Z + o * (int64_t)J;
  for (uint32_t q = threadIdx.x; q < J; q += 256) out[q] = (WT)acc[q];
}

// Y_k (k >= m) from Z.  The outer tuples with i_k = c are o = a + A (c + n_k
// b): a over modes m..k-1 (A tuples, keys KA), b over modes k+1..d-1 (B
// tuples, keys KB).  Workgroup (s, c) adds, for the tuples m = a + A b of
// slice s of the A B, row o of Z shifted cyclically by the bucket of
// key_add(KA[a], KB[b]) and with its sign, into J FP64 LDS entries (thread t
// owns entries t, t + 256, ...: no atomics), and writes them as partial s of
// column c.  Two rows at a time, four entries per thread per load batch.
template <typename WT>
__global__ __launch_bounds__(256) void k_sketch_y_zi(const WT* __restrict__ Z, const uint32_t* __restrict__ KA,
                                                     const uint32_t* __restrict__ KB, double* __restrict__ part,
                                                     int64_t A, int32_t nk, int64_t B, uint32_t J, int32_t S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  typedef const WT __attribute__((address_space(1)))* gwt;
  const int s = blockIdx.x, c = blockIdx.y;
  for (uint32_t q = threadIdx.x; q < J; q += 256) acc[q] = 0.0;   // thread-owned entries
  const int64_t M = A * B;
  const int64_t m0 = (int64_t)s * M / S, m1 = (int64_t)(s + 1) * M / S;
  for (int64_t m = m0; m < m1; m += 2) {
    const bool two = m + 1 < m1;
    const int64_t b0 = m / A, a0 = m - b0 * A;
    const int64_t mm = two ? m + 1 : m;
    const int64_t b1 = mm / A, a1 = mm - b1 * A;
    const uint32_t key0 = key_add(KA[a0], KB[b0], J), key1 = key_add(KA[a1], KB[b1], J);
    const uint32_t h0 = key0 & TT_KEY_MASK, h1 = key1 & TT_KEY_MASK;
    const uint32_t sg0 = key0 & TT_KEY_SIGN, sg1 = two ? (key1 & TT_KEY_SIGN) : 0u;
    const gwt row0 = (gwt)(Z + (a0 + A * (c + (int64_t)nk * b0)) * (int64_t)J);
    const gwt row1 = (gwt)(Z + (a1 + A * (c + (int64_t)nk * b1)) * (int64_t)J);
    for (uint32_t q0 = threadIdx.x; q0 < J; q0 += 256 * 4) {
      WT x0[4], x1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t q = q0 + 256 * u;
        const bool ok = q < J;
        const uint32_t s0 = q >= h0 ? q - h0 : q + J - h0;
        const uint32_t s1 = q >= h1 ? q - h1 : q + J - h1;
        x0[u] = ok ? row0[s0] : WT(0);
        x1[u] = ok && two ? row1[s1] : WT(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t q = q0 + 256 * u;
        if (q < J) acc[q] += signed_f64(x0[u], sg0) + signed_f64(x1[u], sg1);
      }
    }
  }
  double* out = part + ((int64_t)c * S + s) * (int64_t)J;
  for (uint32_t q = threadIdx.x; q < J; q += 256) out[q] = acc[q];
}

// ---------------------------------------------------------------- outer and inner sketch in one pass
// For FP32 work: workgroup w (1024 threads) takes bucket c = order[w] (the
// buckets by number of outer tuples, largest first, so that the last
// workgroups of the launch are short) and reads the whole slabs of the
// outer tuples of key c (the bucket list of the k = 0 sketch), once each,
// and forms from them both
//  * row c of the outer sketch: the slabs summed with their signs, thread t
//    keeping slab positions V (t + 1024 j) + e (j < NV) in FP32 registers;
//  * row o of the inner sketch Z for every slab o of the list: each entry
//    added, with sign v_0(i_0) v_1(i_1), to bucket (h_0(i_0) + h_1(i_1))
//    mod J of a J-entry FP64 LDS array.  A vector's V values share i_1
//    (n_0 is a multiple of V), found as the high word of position times
//    mdiv = ceil(2^32 / n_0) (exact for positions below 2^17); the table
//    entries are read from LDS.
// A slab is read in four chunks of NV / 4 vectors per thread (rounded down or
// up, balanced: 2, 3, 2, 3 for NV = 10); the next
// chunk (of this slab or the next) is loaded before the current one is
// added.  Slabs go in groups of G to G LDS arrays each, two sets alternating
// between groups: after the barrier that closes a group, each thread writes
// its entries of the group's arrays as their rows of Z and clears them while
// the next group goes to the other set, so one barrier per G slabs
// suffices.
template <typename XT, int V, int NV, int G>
__global__ __launch_bounds__(1024) void k_sketch_zoi(const XT* __restrict__ X, const uint32_t* __restrict__ off,
                                                    const uint32_t* __restrict__ sorted,
                                                    const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ tab0, const uint32_t* __restrict__ tab1,
                                                    float* __restrict__ zo, float* __restrict__ Z, int32_t n0,
                                                    int32_t n1, uint32_t J, uint32_t mdiv) {
  constexpr int CH = (NV + 3) / 4;   // most vectors per thread in a chunk (chunk c: j in [c NV / 4, (c + 1) NV / 4))
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);                  // 2 G J entries
  uint32_t* t0 = reinterpret_cast<uint32_t*>(acc + 2 * G * (size_t)J);   // n_0 entries
  uint32_t* t1 = t0 + n0;                                              // n_1 entries
  const int t = threadIdx.x;
  const uint32_t c = order[blockIdx.x];
  const int S = n0 * n1;
  for (uint32_t q = t; q < 2 * G * J; q += 1024) acc[q] = 0.0;
  for (int q = t; q < n0; q += 1024) t0[q] = tab0[q];
  for (int q = t; q < n1; q += 1024) t1[q] = tab1[q];
  float za[NV][V];
#pragma unroll
  for (int j = 0; j < NV; ++j)
#pragma unroll
    for (int e = 0; e < V; ++e) za[j][e] = 0.0f;
  const uint32_t beg = off[c], end = off[c + 1];
  __syncthreads();
  Vec<XT, V> xc[CH], xn[CH];
  auto load_chunk = [&](Vec<XT, V>* x, const XT* slab, int ch) {
#pragma unroll
    for (int h = 0; h < CH; ++h) {
      const int j = ch * NV / 4 + h;
      const int pos = V * (t + 1024 * j);
      if (h < (ch + 1) * NV / 4 - ch * NV / 4 && pos < S) {
        x[h] = load_vec_plain<XT, V>(slab + pos);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) x[h].e[e] = XT(0);
      }
    }
  };
  auto add_chunk = [&](const Vec<XT, V>* x, int ch, double* A, uint32_t so) {
#pragma unroll
    for (int h = 0; h < CH; ++h) {
      const int j = ch * NV / 4 + h;
      if (h >= (ch + 1) * NV / 4 - ch * NV / 4) continue;
      const uint32_t pos = V * (t + 1024 * j);
      if (pos >= (uint32_t)S) continue;
      const uint32_t i1 = __umulhi(pos, mdiv), i0 = pos - i1 * (uint32_t)n0;
      const uint32_t K = t1[i1];
      // the vector's V mode-0 entries in 16-byte LDS reads (t0 and i0 are
      // 16-byte aligned: t0 follows 2 G J doubles, i0 is a multiple of V)
      uint32_t k0v[V];
#pragma unroll
      for (int q = 0; q < V; q += 4) {
        const uint4 w = *reinterpret_cast<const uint4*>(t0 + i0 + q);
        k0v[q] = w.x;
        k0v[q + 1] = w.y;
        k0v[q + 2] = w.z;
        k0v[q + 3] = w.w;
      }
#pragma unroll
      for (int e = 0; e < V; ++e) {
        za[j][e] += __uint_as_float(__float_as_uint(to_work<float>(x[h].e[e])) ^ so);
        const uint32_t b = key_add(k0v[e], K, J);
        atomicAdd(&A[b & TT_KEY_MASK], signed_f64(x[h].e[e], b & TT_KEY_SIGN));
      }
    }
  };
  int buf = 0, np = 0;
  int64_t pend[G];   // Z rows of the group's slabs
  if (beg < end) load_chunk(xc, X + (int64_t)(sorted[beg] & TT_KEY_MASK) * S, 0);
  for (uint32_t it = beg; it < end; ++it) {
    const uint32_t item = sorted[it];
    const int64_t o = item & TT_KEY_MASK;
    const uint32_t so = item & TT_KEY_SIGN;
    const XT* slab = X + o * S;
    const XT* next = it + 1 < end ? X + (int64_t)(sorted[it + 1] & TT_KEY_MASK) * S : nullptr;
    double* A = acc + (size_t)(buf * G + np) * J;
    // chunks 0..3 alternate between the two buffers; chunk 0 of the next
    // slab lands in xc again
    load_chunk(xn, slab, 1);
    add_chunk(xc, 0, A, so);
    load_chunk(xc, slab, 2);
    add_chunk(xn, 1, A, so);
    load_chunk(xn, slab, 3);
    add_chunk(xc, 2, A, so);
    if (next) load_chunk(xc, next, 0);
    add_chunk(xn, 3, A, so);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (g == np) pend[g] = o;
    ++np;
    if (np == G || it + 1 == end) {   // the same for every thread of the workgroup
      __syncthreads();
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g >= np) break;
        double* Ag = acc + (size_t)(buf * G + g) * J;
        float* zr = Z + pend[g] * (int64_t)J;
        for (uint32_t q = t; q < J; q += 1024) {
          zr[q] = (float)Ag[q];
          Ag[q] = 0.0;
        }
      }
      buf ^= 1;
      np = 0;
    }
  }
  float* out = zo + (int64_t)c * S;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int pos = V * (t + 1024 * j);
    if (pos < S) {
#pragma unroll
      for (int e = 0; e < V; ++e) out[pos + e] = za[j][e];
    }
  }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int ilog2_ceil(int64_t x) {
  int l = 0;
  while (((int64_t)1 << l) < x) ++l;
  return l;
}

int g_num_cus = 0;
int num_cus() {
  if (g_num_cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      g_num_cus = n;
    else
      g_num_cus = 256;
  }
  return g_num_cus;
}

template <typename XT, typename WT, int V, int NJ>
hipError_t run_modek(const tt_plan_s* p, const XT* X, int k, WT* Y, int lpf_log2) {
  constexpr int U = NJ >= 8 ? 1 : 8 / NJ;
  const int64_t n0 = p->n[0], nk = p->n[k];
  int64_t M = 1, Rk = 1;
  for (int s = 1; s < k; ++s) M *= p->n[s];
  for (int s = k + 1; s < p->d; ++s) Rk *= p->n[s];
  const int64_t F = M * Rk;
  uint32_t* KI = p->at<uint32_t>(p->o_KI);
  uint32_t* KO = p->at<uint32_t>(p->o_KO);
  hipError_t e;
  {
    TTProfScope ps(p, TT_PROF_SKETCH_AUX);
    // an empty mode range yields the single key 0 (bucket 0, sign +)
    if ((e = launch_build_keys(p, KI, M, 1, k - 1)) != hipSuccess) return e;
    if ((e = launch_build_keys(p, KO, Rk, k + 1, p->d - 1)) != hipSuccess) return e;
  }
  const size_t lds = (size_t)p->J * sizeof(double);
  auto kern = k_sketch_modek<XT, WT, V, NJ, U>;
  int per_cu = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, TT_SKETCH_THREADS, lds)) != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int64_t W = tt_sketch_workgroups(p, k, (int64_t)per_cu * (p->sketch_cus > 0 ? p->sketch_cus : num_cus()));
  const int64_t maxslots = tt_sketch_slots(p, k, W);
  if (nk * maxslots * p->J > p->part_entries) return hipErrorInvalidValue;   // sized at plan time
  double* part = p->at<double>(p->o_part);
  const uint32_t* tab0 = p->at<uint32_t>(p->o_tab) + p->tab_off[0];
  {
    TTProfScope ps(p, TT_PROF_SKETCHK);
    hipLaunchKernelGGL(kern, dim3((unsigned)W), dim3(TT_SKETCH_THREADS), lds, p->stream, X, tab0, KI, KO, part, (int32_t)n0,
                       (int32_t)nk, M, F, (uint32_t)p->J, lpf_log2, (int32_t)maxslots);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  TTProfScope ps(p, TT_PROF_SKETCH_AUX);
  hipLaunchKernelGGL((k_reduce_parts<WT>), dim3(nblk(p->J * nk, 256)), dim3(256), 0, p->stream, part, Y, p->J, nk, F,
                     W, (int32_t)maxslots);
  return hipGetLastError();
}

template <typename XT, typename WT, int V, int NJ>
hipError_t run_gs(const tt_plan_s* p, const XT* X, int k, WT* Y, int lpf_log2) {
  constexpr int U = NJ >= 4 ? 1 : 4 / NJ;
  const int64_t n0 = p->n[0], nk = p->n[k];
  int64_t M = 1, Rk = 1;
  for (int s = 1; s < k; ++s) M *= p->n[s];
  for (int s = k + 1; s < p->d; ++s) Rk *= p->n[s];
  const int64_t F = M * Rk;
  hipError_t e;
  {
    TTProfScope ps(p, TT_PROF_SKETCH_AUX);
    if (!p->lists_ready && (e = launch_fibre_sort(p, k)) != hipSuccess) return e;
  }
  const size_t lds = (size_t)p->J * sizeof(double);
  auto kern = lpf_log2 == 6 ? k_sketch_gs<XT, WT, V, NJ, U, true> : k_sketch_gs<XT, WT, V, NJ, U, false>;
  int per_cu = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, TT_SKETCH_THREADS, lds)) != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int64_t W = tt_sketch_workgroups(p, k, (int64_t)per_cu * (p->sketch_cus > 0 ? p->sketch_cus : num_cus()));
  const int64_t maxslots = tt_sketch_slots(p, k, W);
  if (nk * maxslots * p->J > p->part_entries) return hipErrorInvalidValue;   // sized at plan time
  double* part = p->at<double>(p->o_part);
  const uint32_t* tab0 = p->at<uint32_t>(p->o_tab) + p->tab_off[0];
  {
    TTProfScope ps(p, TT_PROF_SKETCHK);
    hipLaunchKernelGGL(kern, dim3((unsigned)W), dim3(TT_SKETCH_THREADS), lds, p->stream, X, tab0,
                       tt_fibre_list(p, k), part, (int32_t)n0, (int32_t)nk, M, F, (uint32_t)p->J, lpf_log2,
                       (int32_t)maxslots);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  TTProfScope ps(p, TT_PROF_SKETCH_AUX);
  hipLaunchKernelGGL((k_reduce_parts<WT>), dim3(nblk(p->J * nk, 256)), dim3(256), 0, p->stream, part, Y, p->J, nk, F,
                     W, (int32_t)maxslots);
  return hipGetLastError();
}

template <typename XT, typename WT, int V, int NJ>
hipError_t run_mode0(const tt_plan_s* p, const XT* X, WT* Y, int lpf_log2, int64_t chunk) {
  constexpr int U = NJ >= 4 ? 1 : 4 / NJ;
  hipError_t e;
  {
    TTProfScope ps(p, TT_PROF_SKETCH_AUX);
    if (!p->lists_ready && (e = launch_outer_sort(p)) != hipSuccess) return e;
  }
  const int64_t n0 = p->n[0], n1 = p->n[1];
  const uint32_t* tab1 = p->at<uint32_t>(p->o_tab) + p->tab_off[1];
  const uint32_t* off = p->at<uint32_t>(p->o_cnt);
  const uint32_t* sorted = p->at<uint32_t>(p->o_sortO);
  const size_t lds = (size_t)4 * 64 * NJ * V * sizeof(double);
  TTProfScope ps(p, TT_PROF_SKETCH0);
  for (int64_t lo = 0; lo < n0; lo += chunk) {
    const int64_t cnt = (n0 - lo) < chunk ? (n0 - lo) : chunk;
    hipLaunchKernelGGL((k_sketch_mode0<XT, WT, V, NJ, U>), dim3((unsigned)p->J), dim3(256), lds, p->stream, X, tab1, off,
                       sorted, Y, (int32_t)n0, (int32_t)n1, (uint32_t)p->J, (int32_t)lo, (int32_t)cnt, lpf_log2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename WT>
hipError_t launch_y0_zo(const tt_plan_s* p, const WT* zo, WT* Y);

// The fused k = 0 pass: the outer sketch from the slabs (V-value loads when
// n_0 n_1 and the address of X allow), then Y_0 from it.
template <typename XT, typename WT, int V>
hipError_t run_zo_v(const tt_plan_s* p, const XT* X, WT* Y, WT* zo) {
  constexpr int MV = 16 / V;
  const int64_t n0 = p->n[0], n1 = p->n[1], S = n0 * n1, Sv = S / V;
  const int64_t pieces = Sv <= 128 * MV ? 1 : (Sv + 256 * MV - 1) / (256 * MV);
  const uint32_t* off = p->at<uint32_t>(p->o_cnt);
  const uint32_t* sorted = p->at<uint32_t>(p->o_sortO);
  hipLaunchKernelGGL((k_sketch_zo<XT, WT, V, MV, 2>), dim3((unsigned)pieces, (unsigned)p->J), dim3(256), 0, p->stream,
                     X, off, sorted, zo, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_y0_zo<WT>(p, zo, Y);
}

// Y_0 from the outer sketch (k_sketch_y0_zo), one workgroup per bucket.
template <typename WT>
hipError_t launch_y0_zo(const tt_plan_s* p, const WT* zo, WT* Y) {
  const int64_t n0 = p->n[0], n1 = p->n[1];
  const uint32_t* tab1 = p->at<uint32_t>(p->o_tab) + p->tab_off[1];
  const dim3 g((unsigned)p->J);
  const int32_t a0 = (int32_t)n0, a1 = (int32_t)n1;
  const uint32_t J = (uint32_t)p->J;
  if (n0 <= 256) hipLaunchKernelGGL((k_sketch_y0_zo<WT, 1>), g, dim3(256), 0, p->stream, zo, tab1, Y, a0, a1, J);
  else if (n0 <= 512) hipLaunchKernelGGL((k_sketch_y0_zo<WT, 2>), g, dim3(256), 0, p->stream, zo, tab1, Y, a0, a1, J);
  else if (n0 <= 1024) hipLaunchKernelGGL((k_sketch_y0_zo<WT, 4>), g, dim3(256), 0, p->stream, zo, tab1, Y, a0, a1, J);
  else if (n0 <= 2048) hipLaunchKernelGGL((k_sketch_y0_zo<WT, 8>), g, dim3(256), 0, p->stream, zo, tab1, Y, a0, a1, J);
  else if (n0 <= 4096) hipLaunchKernelGGL((k_sketch_y0_zo<WT, 16>), g, dim3(256), 0, p->stream, zo, tab1, Y, a0, a1, J);
  else return hipErrorInvalidValue;   // not reached: plans take n_0 <= TT_MAX_N0 = 4096
  return hipGetLastError();
}

// The one pass for the outer and the inner sketch (FP32 work), then Y_0.
// order[] = the J buckets by their number of outer tuples (off[c + 1] -
// off[c], counted up to 255), largest first; one workgroup.  The order
// within a count follows LDS atomics and does not affect any result.
__global__ __launch_bounds__(1024) void k_bucket_order(const uint32_t* __restrict__ off, uint32_t* __restrict__ order,
                                                       uint32_t J) {
  __shared__ uint32_t hist[256];
  const int t = threadIdx.x;
  if (t < 256) hist[t] = 0;
  __syncthreads();
  for (uint32_t c = t; c < J; c += 1024) {
    const uint32_t n = off[c + 1] - off[c];
    atomicAdd(&hist[255 - (n < 255 ? n : 255)], 1u);
  }
  __syncthreads();
  if (t == 0) {   // exclusive prefix sum: bin 0 holds the largest buckets
    uint32_t run = 0;
    for (int b = 0; b < 256; ++b) {
      const uint32_t h = hist[b];
      hist[b] = run;
      run += h;
    }
  }
  __syncthreads();
  for (uint32_t c = t; c < J; c += 1024) {
    const uint32_t n = off[c + 1] - off[c];
    order[atomicAdd(&hist[255 - (n < 255 ? n : 255)], 1u)] = c;
  }
}

template <typename XT, int NV>
hipError_t run_zoi_v(const tt_plan_s* p, const XT* X, float* Y, float* zo) {
  constexpr int V = 16 / (int)sizeof(XT);
  const size_t tabs = (size_t)(p->n[0] + p->n[1]) * sizeof(uint32_t);
  // two slabs per barrier when four bucket arrays fit in LDS
  const bool two = 4 * (size_t)p->J * sizeof(double) + tabs <= 160 * 1024;
  const size_t lds = (two ? 4 : 2) * (size_t)p->J * sizeof(double) + tabs;
  auto kern = two ? k_sketch_zoi<XT, V, NV, 2> : k_sketch_zoi<XT, V, NV, 1>;
  hipError_t e;
  if ((e = tt_allow_lds(kern, lds)) != hipSuccess) return e;
  const uint32_t* tab = p->at<uint32_t>(p->o_tab);
  uint32_t* order = p->at<uint32_t>(p->o_zperm);
  hipLaunchKernelGGL(k_bucket_order, dim3(1), dim3(1024), 0, p->stream, p->at<uint32_t>(p->o_cnt), order,
                     (uint32_t)p->J);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)p->J), dim3(1024), lds, p->stream, X, p->at<uint32_t>(p->o_cnt),
                     p->at<uint32_t>(p->o_sortO), order, tab + p->tab_off[0], tab + p->tab_off[1], zo,
                     p->at<float>(p->o_zi),
                     (int32_t)p->n[0], (int32_t)p->n[1], (uint32_t)p->J,
                     (uint32_t)((((uint64_t)1 << 32) + (uint64_t)p->n[0] - 1) / (uint64_t)p->n[0]));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_y0_zo<float>(p, zo, Y);
}

template <typename XT>
hipError_t run_zoi(const tt_plan_s* p, const XT* X, float* Y, float* zo) {
  const int nv = tt_joint_vectors(p);
  if constexpr (sizeof(XT) == 2) {   // BF16: 4 vectors of 8 values
    if (nv == 4) return run_zoi_v<XT, 4>(p, X, Y, zo);
  } else {
    if (nv == 4) return run_zoi_v<XT, 4>(p, X, Y, zo);
    if (nv == 8) return run_zoi_v<XT, 8>(p, X, Y, zo);
    if (nv == 10) return run_zoi_v<XT, 10>(p, X, Y, zo);
  }
  return hipErrorInvalidValue;   // not reached: the plan takes the path for these counts only
}

template <typename XT, typename WT>
hipError_t run_zo(const tt_plan_s* p, const XT* X, WT* Y, WT* zo) {
  hipError_t e;
  {
    TTProfScope ps(p, TT_PROF_SKETCH_AUX);
    if (!p->lists_ready && (e = launch_outer_sort(p)) != hipSuccess) return e;
  }
  TTProfScope ps(p, TT_PROF_SKETCH0);
  if constexpr (std::is_same<WT, float>::value && !std::is_same<XT, double>::value) {
    if (tt_sketch_joint_ok(p, X)) return run_zoi<XT>(p, X, Y, zo);
  }
  constexpr int VV = 16 / (int)sizeof(XT);
  const bool vec = (p->n[0] * p->n[1]) % VV == 0 && ((uintptr_t)X % 16) == 0;
  return vec ? run_zo_v<XT, WT, VV>(p, X, Y, zo) : run_zo_v<XT, WT, 1>(p, X, Y, zo);
}

// Lanes per fibre (power of two <= 64) and vector loads per lane for n0.
void lane_shape(int64_t n0, int V, int* lpf_log2, int* nj) {
  const int64_t vecs = (n0 + V - 1) / V;
  if (vecs <= 64) {
    *lpf_log2 = ilog2_ceil(vecs);
    *nj = 1;
  } else {
    *lpf_log2 = 6;
    *nj = 1 << ilog2_ceil((vecs + 63) / 64);
  }
}

template <typename XT, typename WT, int V>
hipError_t dispatch_v(const tt_plan_s* p, const XT* X, int k, WT* Y, WT* zo) {
  const int64_t n0 = p->n[0];
  int lpf, nj;
  if (k == 0) {
    if (zo) return run_zo<XT, WT>(p, X, Y, zo);
    // the k = 0 gather covers at most 64 * 4 * V positions of i_0 per launch
    const int64_t chunk = 64 * 4 * V;
    lane_shape(n0 < chunk ? n0 : chunk, V, &lpf, &nj);
    switch (nj) {
      case 1: return run_mode0<XT, WT, V, 1>(p, X, Y, lpf, chunk);
      case 2: return run_mode0<XT, WT, V, 2>(p, X, Y, lpf, chunk);
      default: return run_mode0<XT, WT, V, 4>(p, X, Y, lpf, chunk);
    }
  }
  lane_shape(n0, V, &lpf, &nj);
  if (tt_sketch_use_gs(p, k)) {
    switch (nj) {
      case 1: return run_gs<XT, WT, V, 1>(p, X, k, Y, lpf);
      case 2: return run_gs<XT, WT, V, 2>(p, X, k, Y, lpf);
      case 4: return run_gs<XT, WT, V, 4>(p, X, k, Y, lpf);
      case 8: return run_gs<XT, WT, V, 8>(p, X, k, Y, lpf);
      case 16: return run_gs<XT, WT, V, 16>(p, X, k, Y, lpf);
      case 32: return run_gs<XT, WT, V, 32>(p, X, k, Y, lpf);
      default: return run_gs<XT, WT, V, 64>(p, X, k, Y, lpf);
    }
  }
  switch (nj) {
    case 1: return run_modek<XT, WT, V, 1>(p, X, k, Y, lpf);
    case 2: return run_modek<XT, WT, V, 2>(p, X, k, Y, lpf);
    case 4: return run_modek<XT, WT, V, 4>(p, X, k, Y, lpf);
    case 8: return run_modek<XT, WT, V, 8>(p, X, k, Y, lpf);
    case 16: return run_modek<XT, WT, V, 16>(p, X, k, Y, lpf);
    case 32: return run_modek<XT, WT, V, 32>(p, X, k, Y, lpf);
    default: return run_modek<XT, WT, V, 64>(p, X, k, Y, lpf);
  }
}

template <typename XT, typename WT>
hipError_t dispatch(const tt_plan_s* p, const void* Xv, int k, void* Yv, void* zov) {
  const XT* X = static_cast<const XT*>(Xv);
  WT* Y = static_cast<WT*>(Yv);
  WT* zo = static_cast<WT*>(zov);
  constexpr int VV = 16 / (int)sizeof(XT);
  // 16-byte loads when every fibre starts on a 16-byte boundary
  const bool vec = (p->n[0] % VV) == 0 && ((uintptr_t)Xv % 16) == 0;
  return vec ? dispatch_v<XT, WT, VV>(p, X, k, Y, zo) : dispatch_v<XT, WT, 1>(p, X, k, Y, zo);
}

template <typename WT>
hipError_t run_y1_outer(const tt_plan_s* p, void* Yv) {
  const int64_t n0 = p->n[0], n1 = p->n[1];
  const int S = (int)tt_outer_slices(p);
  double* part = p->at<double>(p->o_part);
  if (n1 * S * p->J > p->part_entries) return hipErrorInvalidValue;   // sized at plan time
  const size_t lds = (size_t)((p->J + 1) & ~(int64_t)1) * sizeof(double) + (size_t)n0 * sizeof(uint32_t);
  // 16-byte loads when every row of n_0 values starts on a 16-byte boundary
  constexpr int VW = 16 / (int)sizeof(WT);
  auto kern = (n0 % VW) == 0 ? k_sketch_y1_outer<WT, VW> : k_sketch_y1_outer<WT, 1>;
  hipError_t e;
  if ((e = tt_allow_lds(kern, lds)) != hipSuccess) return e;
  const uint32_t* tab = p->at<uint32_t>(p->o_tab);
  {
    TTProfScope ps(p, TT_PROF_SKETCH_AUX);
    hipLaunchKernelGGL(kern, dim3((unsigned)S, (unsigned)n1), dim3(256), lds, p->stream, p->at<WT>(p->o_zo),
                       tab + p->tab_off[0], part, (int32_t)n0, (int32_t)n1, (uint32_t)p->J, S);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  TTProfScope ps(p, TT_PROF_SKETCH_AUX);
  hipLaunchKernelGGL(k_reduce_slots<WT>, dim3(nblk(p->J * n1, 256)), dim3(256), 0, p->stream, part,
                     static_cast<WT*>(Yv), p->J, n1, S);
  return hipGetLastError();
}

// The inner-sketch pass: Z from X, one workgroup per outer tuple.
template <typename XT, typename WT, int V, int NJ>
hipError_t run_zi_v(const tt_plan_s* p, const XT* X, WT* Z, int lpf_log2) {
  constexpr int U = NJ >= 4 ? 1 : 4 / NJ;
  const size_t lds = (size_t)p->J * sizeof(double) + (size_t)p->inner_rows * sizeof(uint32_t);
  auto kern = k_sketch_zi<XT, WT, V, NJ, U>;
  hipError_t e;
  if ((e = tt_allow_lds(kern, lds)) != hipSuccess) return e;
  const uint32_t* tab = p->at<uint32_t>(p->o_tab);
  // row keys: the mode-1 table when m = 2, else the keys over modes 1..m-1
  const uint32_t* rkey = tab + p->tab_off[1];
  if (p->inner_m > 2) {
    uint32_t* KR = p->at<uint32_t>(p->o_KI);
    if ((e = launch_build_keys(p, KR, p->inner_rows, 1, p->inner_m - 1)) != hipSuccess) return e;
    rkey = KR;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)p->inner_O), dim3(256), lds, p->stream, X, tab + p->tab_off[0], rkey, Z,
                     (int32_t)p->n[0], (int32_t)p->inner_rows, (uint32_t)p->J, lpf_log2);
  return hipGetLastError();
}

template <typename XT, typename WT, int V>
hipError_t run_zi_shape(const tt_plan_s* p, const XT* X, WT* Z) {
  int lpf, nj;
  lane_shape(p->n[0], V, &lpf, &nj);
  switch (nj) {
    case 1: return run_zi_v<XT, WT, V, 1>(p, X, Z, lpf);
    case 2: return run_zi_v<XT, WT, V, 2>(p, X, Z, lpf);
    case 4: return run_zi_v<XT, WT, V, 4>(p, X, Z, lpf);
    case 8: return run_zi_v<XT, WT, V, 8>(p, X, Z, lpf);
    case 16: return run_zi_v<XT, WT, V, 16>(p, X, Z, lpf);
    default: return hipErrorInvalidValue;   // not reached: the plan takes this path for n_0 <= 1024 only
  }
}

template <typename XT, typename WT>
hipError_t run_zi(const tt_plan_s* p, const void* Xv) {
  const XT* X = static_cast<const XT*>(Xv);
  WT* Z = p->at<WT>(p->o_zi);
  constexpr int VV = 16 / (int)sizeof(XT);
  const bool vec = (p->n[0] % VV) == 0 && ((uintptr_t)Xv % 16) == 0;
  return vec ? run_zi_shape<XT, WT, VV>(p, X, Z) : run_zi_shape<XT, WT, 1>(p, X, Z);
}

// Y_k (k >= 2) from Z: keys of the modes 2..k-1 and k+1..d-1, the partials,
// their sum.
template <typename WT>
hipError_t run_y_inner(const tt_plan_s* p, int k, void* Yv) {
  int64_t A = 1, B = 1;
  for (int s = p->inner_m; s < k; ++s) A *= p->n[s];
  for (int s = k + 1; s < p->d; ++s) B *= p->n[s];
  const int64_t nk = p->n[k];
  const int S = (int)tt_inner_slices(p, k);
  if (nk * S * p->J > p->part_entries) return hipErrorInvalidValue;   // sized at plan time
  uint32_t* KA = p->at<uint32_t>(p->o_KI);
  uint32_t* KB = p->at<uint32_t>(p->o_KO);
  double* part = p->at<double>(p->o_part);
  hipError_t e;
  // an empty mode range yields the single key 0 (bucket 0, sign +)
  if ((e = launch_build_keys(p, KA, A, p->inner_m, k - 1)) != hipSuccess) return e;
  if ((e = launch_build_keys(p, KB, B, k + 1, p->d - 1)) != hipSuccess) return e;
  const size_t lds = (size_t)p->J * sizeof(double);
  if ((e = tt_allow_lds(k_sketch_y_zi<WT>, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sketch_y_zi<WT>, dim3((unsigned)S, (unsigned)nk), dim3(256), lds, p->stream,
                     p->at<WT>(p->o_zi), KA, KB, part, A, (int32_t)nk, B, (uint32_t)p->J, (int32_t)S);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_slots<WT>, dim3(nblk(p->J * nk, 256)), dim3(256), 0, p->stream, part,
                     static_cast<WT*>(Yv), p->J, nk, S);
  return hipGetLastError();
}

}  // namespace

// Workgroups of the k >= 1 sketch: the occupancy-limited resident count,
// capped so that each workgroup streams at least 8 J entries of X per J-entry
// partial it writes, by the number of fibres (every range non-empty) and by
// TT_SKETCH_MAX_WG.
int64_t tt_sketch_workgroups(const tt_plan_s* p, int k, int64_t resident) {
  const int64_t Ftot = p->N / p->n[0];
  int64_t W = resident;
  const int64_t cap = p->N / (8 * p->J);
  if (W > cap) W = cap;
  if (W > Ftot) W = Ftot;
  if (W > TT_SKETCH_MAX_WG) W = TT_SKETCH_MAX_WG;
  (void)k;
  return W < 1 ? 1 : W;
}

// Upper bound on the workgroups whose ranges meet one column: ranges hold at
// least m = floor(Ftot / W) >= 1 fibres, a column F consecutive fibres.
int64_t tt_sketch_slots(const tt_plan_s* p, int k, int64_t W) {
  const int64_t Ftot = p->N / p->n[0];
  const int64_t F = Ftot / p->n[k];
  const int64_t m = Ftot / W;
  return (F - 1) / m + 2;
}

// Key-grouped path for k >= 1 when a column has at least two fibres per key
// on average and fibre offsets fit the 31-bit list entries.
bool tt_sketch_use_gs(const tt_plan_s* p, int k) {
  if (k < 1) return false;
  const int64_t F = p->N / (p->n[0] * p->n[k]);
  return F >= (int64_t)TT_SKETCH_GS_MIN * p->J && p->N / p->n[0] < ((int64_t)1 << 31);
}

static hipError_t sketch_any(const tt_plan_s* p, const void* X, int k, void* Y, void* zo) {
  if (p->wdt == TT_F64) {
    if (p->xdt == TT_F64) return dispatch<double, double>(p, X, k, Y, zo);
    if (p->xdt == TT_F32) return dispatch<float, double>(p, X, k, Y, zo);
    return dispatch<uint16_t, double>(p, X, k, Y, zo);
  }
  if (p->xdt == TT_F64) return dispatch<double, float>(p, X, k, Y, zo);
  if (p->xdt == TT_F32) return dispatch<float, float>(p, X, k, Y, zo);
  return dispatch<uint16_t, float>(p, X, k, Y, zo);
}

hipError_t launch_sketch_tensor(const tt_plan_s* p, const void* X, int k, void* Y) {
  return sketch_any(p, X, k, Y, nullptr);
}

// Workgroups per column of the Y_1-from-outer-sketch kernel: about 1024 in
// all, and at most n_0 / 4 per column, so that a workgroup reads at least 4 J
// values for the J-entry partial it writes.  Independent of J: partials
// sized for the plan's J hold those of every smaller J.
int64_t tt_outer_slices(const tt_plan_s* p) {
  int64_t S = (1024 + p->n[1] - 1) / p->n[1];
  const int64_t cap = p->n[0] / 4 > 1 ? p->n[0] / 4 : 1;
  if (S > cap) S = cap;
  return S < 1 ? 1 : S;
}

// The fused k = 0 pass writes the outer sketch: d >= 3 and the plan holds
// the J_cap n_0 n_1 buffer for it.
bool tt_sketch_fused01(const tt_plan_s* p) { return p->o_zo != 0; }

hipError_t launch_sketch_mode0_outer(const tt_plan_s* p, const void* X, void* Y0) {
  if (!tt_sketch_fused01(p)) return hipErrorInvalidValue;
  return sketch_any(p, X, 0, Y0, p->ws + p->o_zo);
}

hipError_t launch_sketch_y1_outer(const tt_plan_s* p, void* Y1) {
  if (!tt_sketch_fused01(p)) return hipErrorInvalidValue;
  return p->wdt == TT_F64 ? run_y1_outer<double>(p, Y1) : run_y1_outer<float>(p, Y1);
}

// Workgroups per column of the Y_k-from-Z kernel (k >= 2): about 1024 in all,
// each summing at least 2 rows of Z.
int64_t tt_inner_slices(const tt_plan_s* p, int k) {
  const int64_t M = p->inner_O / p->n[k];
  int64_t S = (1024 + p->n[k] - 1) / p->n[k];
  const int64_t cap = M / 2 > 1 ? M / 2 : 1;
  if (S > cap) S = cap;
  return S < 1 ? 1 : S;
}

// Y_k for k >= inner_m come from the inner sketch Z: the plan holds the
// J_cap x inner_O buffer for it.
bool tt_sketch_inner(const tt_plan_s* p) { return p->o_zi != 0; }

// One pass over X writes Z (the TensorSketch of every slab over modes
// 0..m-1; by the k = 0 pass instead when it writes both intermediates), then
// Y_k for every k >= m is formed from Z into its slot of Yall.
hipError_t launch_sketch_inner(const tt_plan_s* p, const void* X, void* Yall) {
  if (!tt_sketch_inner(p)) return hipErrorInvalidValue;
  hipError_t e;
  if (!tt_sketch_joint_ok(p, X)) {   // else Z was written by the k = 0 pass
    TTProfScope ps(p, TT_PROF_SKETCHK);
    if (p->wdt == TT_F64) {
      e = p->xdt == TT_F64 ? run_zi<double, double>(p, X)
          : p->xdt == TT_F32 ? run_zi<float, double>(p, X) : run_zi<uint16_t, double>(p, X);
    } else {
      e = p->xdt == TT_F64 ? run_zi<double, float>(p, X)
          : p->xdt == TT_F32 ? run_zi<float, float>(p, X) : run_zi<uint16_t, float>(p, X);
    }
    if (e != hipSuccess) return e;
  }
  TTProfScope ps(p, TT_PROF_SKETCH_AUX);
  char* Yb = static_cast<char*>(Yall);
  for (int k = p->inner_m; k < p->d; ++k) {
    void* Yk = Yb + p->wsize() * p->J * p->tab_off[k];
    e = p->wdt == TT_F64 ? run_y_inner<double>(p, k, Yk) : run_y_inner<float>(p, k, Yk);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The k = 0 pass also writes the inner sketch (k_sketch_zoi): FP32 work, FP32
// or BF16 X, both sketches in the plan, rows of whole V-value vectors, at
// most 40 values of a slab per thread (4, 8 or 10 vectors of FP32, 4 of
// BF16: the outer-sketch sums stay in registers), tables and both bucket
// arrays within 160 KB of LDS.
int tt_joint_vectors(const tt_plan_s* p) {
  if (!(tt_sketch_fused01(p) && tt_sketch_inner(p)) || p->inner_m != 2 || p->wdt != TT_F32 || p->xdt == TT_F64)
    return 0;
  const int64_t V = 16 / (int64_t)p->xsize(), S = p->n[0] * p->n[1];
  if (p->n[0] % V != 0 || p->n[0] > 4096) return 0;
  if (16 * p->J_cap + 4 * (p->n[0] + p->n[1]) > 160 * 1024) return 0;
  const int64_t nv = (S / V + 1023) / 1024;
  const int NV = nv <= 4 ? 4 : nv <= 8 ? 8 : 10;
  return nv <= NV && NV * V <= 40 ? NV : 0;
}

bool tt_sketch_joint(const tt_plan_s* p) { return tt_joint_vectors(p) > 0; }

// The joint pass runs when the plan takes it and X is 16-byte aligned (the
// slabs are then read in whole vectors); otherwise the two passes run.
bool tt_sketch_joint_ok(const tt_plan_s* p, const void* X) {
  return tt_sketch_joint(p) && ((uintptr_t)X % 16) == 0;
}
