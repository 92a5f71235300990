// Seeded TensorSketch tables and the derived per-fibre key tables.
//
// Tables (Sec. 2.2, Definitions of CountSketch and TensorSketch; Algorithm 1
// draws new operators once per outer iteration): every entry of h_s and v_s
// is an independent SplitMix64 output (Steele, Lea, Flood 2014), generated
// directly on the device, one thread per entry.
#include "tt_internal.h"

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct TabArgs {
  int32_t off[TT_MAX_ORDER + 1];
  int32_t d;
  uint32_t J;
  uint64_t seed;
  int64_t sweep;
  const int64_t* dsweep;   // if set, the sweep index is read from device memory
};

// tab[off[s] + i] = h_s[i] | (v_s[i] < 0) << 31
__global__ void k_gen_tables(uint32_t* tab, TabArgs a) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.off[a.d]) return;
  int s = 0;
  while (g >= a.off[s + 1]) ++s;
  const uint64_t i = (uint64_t)(g - a.off[s]);
  const uint64_t ns = (uint64_t)(a.off[s + 1] - a.off[s]);
  const int64_t sweep = a.dsweep ? *a.dsweep : a.sweep;
  const uint64_t key = a.seed ^ ((uint64_t)(sweep + 1) * 65536ull + (uint64_t)s);
  const uint64_t st = mix64(key);
  const uint64_t xh = mix64(st + (i + 1) * kGamma);
  const uint64_t xv = mix64(st + (ns + i + 1) * kGamma);
  const uint32_t h = (uint32_t)__umul64hi(xh, (uint64_t)a.J);   // floor(xh * J / 2^64)
  tab[g] = h | ((uint32_t)(xv >> 63) << 31);
}

struct KeyArgs {
  const uint32_t* tab;
  int32_t tab_off[TT_MAX_ORDER];
  int32_t n[TT_MAX_ORDER];
  int32_t modes[TT_MAX_ORDER];   // modes of the tuple, first varies fastest
  int32_t nm;
  uint32_t J;
};

__device__ __forceinline__ uint32_t key_add(uint32_t a, uint32_t b, uint32_t J) {
  uint32_t s = (a & TT_KEY_MASK) + (b & TT_KEY_MASK);
  s = s >= J ? s - J : s;
  return s | ((a ^ b) & TT_KEY_SIGN);
}

// combined key (sum of hashes mod J, product of signs) of tuple q
__device__ __forceinline__ uint32_t tuple_key(uint32_t q, const KeyArgs& a) {
  uint32_t rem = q, key = 0;
  for (int t = 0; t < a.nm; ++t) {
    const int s = a.modes[t];
    const uint32_t nxt = rem / (uint32_t)a.n[s];
    key = key_add(key, a.tab[a.tab_off[s] + (rem - nxt * (uint32_t)a.n[s])], a.J);
    rem = nxt;
  }
  return key;
}

// out[q] = key of tuple q (q < 2^31)
__global__ void k_build_keys(uint32_t* out, int64_t count, KeyArgs a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  out[q] = tuple_key((uint32_t)q, a);
}

// Counting sort of tuple keys by bucket, in three launches and without
// global atomics.  The tuples are cut into nb contiguous chunks.
//  1. k_sort_count: workgroup w computes the keys of chunk w, stores them,
//     counts them per bucket in LDS and writes the counts to hist[w][.].
//  2. k_sort_scan (one workgroup): per bucket b, hist[w][b] becomes the
//     number of earlier-chunk tuples in b; the bucket totals are scanned into
//     off[0..J] (off[J] = number of tuples).
//  3. k_sort_place: chunk w's tuples of bucket b go to positions
//     off[b] + hist[w][b] onward, ranked inside the chunk by LDS atomics.
// The order inside a bucket follows those atomics and is not fixed; the data
// sketches that read the lists sum in FP64, so their output does not show it.
constexpr int kSortThreads = 1024;
constexpr int kSortPerThread = 8;       // tuples per thread and round, loaded before they are used
constexpr int64_t kSortMaxChunks = 64;

__global__ __launch_bounds__(kSortThreads) void k_sort_count(uint32_t* __restrict__ keys, int64_t count, int64_t chunk,
                                                             KeyArgs a, uint32_t* __restrict__ hist) {
  extern __shared__ uint32_t h[];   // J
  for (uint32_t b = threadIdx.x; b < a.J; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < count ? lo + chunk : count;
  for (int64_t q0 = lo + threadIdx.x; q0 < hi; q0 += (int64_t)kSortPerThread * blockDim.x) {
    uint32_t key[kSortPerThread];
#pragma unroll
    for (int u = 0; u < kSortPerThread; ++u) {
      const int64_t q = q0 + (int64_t)u * blockDim.x;
      key[u] = q < hi ? tuple_key((uint32_t)q, a) : 0u;
    }
#pragma unroll
    for (int u = 0; u < kSortPerThread; ++u) {
      const int64_t q = q0 + (int64_t)u * blockDim.x;
      if (q < hi) {
        keys[q] = key[u];
        atomicAdd(&h[key[u] & TT_KEY_MASK], 1u);
      }
    }
  }
  __syncthreads();
  uint32_t* out = hist + (int64_t)blockIdx.x * a.J;
  for (uint32_t b = threadIdx.x; b < a.J; b += blockDim.x) out[b] = h[b];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scan(uint32_t* __restrict__ hist, int32_t nb, int32_t J,
                                                            uint32_t* __restrict__ off) {
  extern __shared__ uint32_t tot[];   // J
  __shared__ uint32_t wsum[kSortThreads / 64];
  const int t = threadIdx.x, T = blockDim.x, lane = t & 63, w = t >> 6, NW = T >> 6;
  constexpr int CB = 16;   // chunk counts loaded together
  for (int b = t; b < J; b += T) {
    uint32_t run = 0;
    for (int c0 = 0; c0 < nb; c0 += CB) {
      uint32_t v[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) v[u] = c0 + u < nb ? hist[(int64_t)(c0 + u) * J + b] : 0u;
#pragma unroll
      for (int u = 0; u < CB; ++u)
        if (c0 + u < nb) {
          hist[(int64_t)(c0 + u) * J + b] = run;
          run += v[u];
        }
    }
    tot[b] = run;
  }
  __syncthreads();
  // exclusive scan of tot: per-thread runs, shuffles within each wave, then
  // over the wave totals
  const int per = (J + T - 1) / T;
  const int lo = min(J, t * per), hi = min(J, lo + per);
  uint32_t s = 0;
  for (int c = lo; c < hi; ++c) s += tot[c];
  uint32_t x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (w == 0) {
    uint32_t v = lane < NW ? wsum[lane] : 0u;
    const uint32_t own = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)v, o, 64);
      if (lane >= o) v += y;
    }
    if (lane < NW) wsum[lane] = v - own;   // exclusive over the waves
  }
  __syncthreads();
  uint32_t acc = wsum[w] + x - s;          // exclusive prefix of this thread's run
  if (t == T - 1) off[J] = acc + s;
  for (int c = lo; c < hi; ++c) {
    off[c] = acc;
    acc += tot[c];
  }
}

// FIBRE: the list of the k >= 1 sketch, tuple t = mu + M rho of a column
// (modes 1..k-1 give mu, modes k+1..d-1 give rho) stored as {column-
// independent fibre offset rho n_k M + mu with the key's sign bit; bucket}.
// Otherwise the k = 0 bucket lists: {t with the key's sign bit}.
template <bool FIBRE>
__global__ __launch_bounds__(kSortThreads) void k_sort_place(const uint32_t* __restrict__ keys, int64_t count,
                                                             int64_t chunk, const uint32_t* __restrict__ hist,
                                                             const uint32_t* __restrict__ off, int32_t J,
                                                             uint32_t* __restrict__ sorted, uint2* __restrict__ fsorted,
                                                             uint32_t M, uint32_t nkM) {
  extern __shared__ uint32_t h[];   // J
  const uint32_t* hw = hist + (int64_t)blockIdx.x * J;
  for (int b = threadIdx.x; b < J; b += blockDim.x) h[b] = off[b] + hw[b];
  __syncthreads();
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < count ? lo + chunk : count;
  for (int64_t q0 = lo + threadIdx.x; q0 < hi; q0 += (int64_t)kSortPerThread * blockDim.x) {
    uint32_t key[kSortPerThread];
#pragma unroll
    for (int u = 0; u < kSortPerThread; ++u) {
      const int64_t q = q0 + (int64_t)u * blockDim.x;
      key[u] = q < hi ? keys[q] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kSortPerThread; ++u) {
      const int64_t q = q0 + (int64_t)u * blockDim.x;
      if (q < hi) {
        const uint32_t c = key[u] & TT_KEY_MASK;
        const uint32_t pos = atomicAdd(&h[c], 1u);
        if constexpr (FIBRE) {
          const uint32_t rho = (uint32_t)q / M, mu = (uint32_t)q - rho * M;
          fsorted[pos] = make_uint2((rho * nkM + mu) | (key[u] & TT_KEY_SIGN), c);
        } else {
          sorted[pos] = (uint32_t)q | (key[u] & TT_KEY_SIGN);
        }
      }
    }
  }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_gen_tables(const tt_plan_s* p, int64_t sweep) {
  TabArgs a{};
  for (int s = 0; s <= p->d; ++s) a.off[s] = (int32_t)p->tab_off[s];
  a.d = p->d;
  a.J = (uint32_t)p->J;
  a.seed = p->seed;
  a.sweep = sweep;
  a.dsweep = p->dsweep;
  const int64_t total = p->tab_off[p->d];
  hipLaunchKernelGGL(k_gen_tables, dim3(nblk(total, 256)), dim3(256), 0, p->stream,
                     p->at<uint32_t>(p->o_tab), a);
  return hipGetLastError();
}

int64_t tt_sort_chunks(int64_t count) {
  const int64_t per = (int64_t)kSortPerThread * kSortThreads;   // one round of tuples per workgroup
  int64_t nb = (count + per - 1) / per;
  return nb < 1 ? 1 : (nb > kSortMaxChunks ? kSortMaxChunks : nb);
}

namespace {

KeyArgs key_args(const tt_plan_s* p, const int* modes, int nm) {
  KeyArgs a{};
  a.tab = p->at<uint32_t>(p->o_tab);
  for (int s = 0; s < p->d; ++s) {
    a.tab_off[s] = (int32_t)p->tab_off[s];
    a.n[s] = (int32_t)p->n[s];
  }
  for (int t = 0; t < nm; ++t) a.modes[t] = modes[t];
  a.nm = nm;
  a.J = (uint32_t)p->J;
  return a;
}

// keys (count entries) and the J+1 offsets of the sort of `count` tuples
hipError_t sort_keys(const tt_plan_s* p, const int* modes, int nm, int64_t count, uint32_t* keys, uint32_t* off,
                     int64_t* nb_out, int64_t* chunk_out) {
  if (count < 1 || count >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int64_t nb = tt_sort_chunks(count), chunk = (count + nb - 1) / nb;
  uint32_t* hist = p->at<uint32_t>(p->o_hist);
  const size_t lds = sizeof(uint32_t) * p->J;
  hipLaunchKernelGGL(k_sort_count, dim3((unsigned)nb), dim3(kSortThreads), lds, p->stream, keys, count, chunk,
                     key_args(p, modes, nm), hist);
  hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kSortThreads), lds, p->stream, hist, (int32_t)nb, (int32_t)p->J, off);
  *nb_out = nb;
  *chunk_out = chunk;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_build_keys_modes(const tt_plan_s* p, uint32_t* out, int64_t count, const int* modes, int nm) {
  if (count <= 0) return hipSuccess;
  if (count >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_build_keys, dim3(nblk(count, 256)), dim3(256), 0, p->stream, out, count, key_args(p, modes, nm));
  return hipGetLastError();
}

hipError_t launch_build_keys(const tt_plan_s* p, uint32_t* out, int64_t count, int first, int last) {
  int modes[TT_MAX_ORDER];
  int nm = 0;
  for (int s = first; s <= last; ++s) modes[nm++] = s;
  return launch_build_keys_modes(p, out, count, modes, nm);
}

// Bucket lists of the k = 0 data sketch: the outer mode tuples (modes
// 2..d-1) grouped by their partial hash.  Uses o_KO as key scratch.
hipError_t launch_outer_sort(const tt_plan_s* p) {
  const int64_t O = p->O0;
  int modes[TT_MAX_ORDER];
  int nm = 0;
  for (int s = 2; s < p->d; ++s) modes[nm++] = s;
  uint32_t* keys = p->at<uint32_t>(p->o_KO);
  uint32_t* off = p->at<uint32_t>(p->o_cnt);          // J+1
  int64_t nb = 0, chunk = 0;
  hipError_t e = sort_keys(p, modes, nm, O, keys, off, &nb, &chunk);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sort_place<false>, dim3((unsigned)nb), dim3(kSortThreads), sizeof(uint32_t) * p->J, p->stream,
                     keys, O, chunk, p->at<uint32_t>(p->o_hist), off, (int32_t)p->J, p->at<uint32_t>(p->o_sortO),
                     (uint2*)nullptr, 1u, 1u);
  return hipGetLastError();
}

// Sort the fibres of a mode-k column (k >= 1) by their key over modes != 0, k.
// Offsets of the J buckets go to o_cnt (J+1 entries), the list to o_fsort.
hipError_t launch_fibre_sort(const tt_plan_s* p, int k) {
  int64_t M = 1, Rk = 1;
  for (int s = 1; s < k; ++s) M *= p->n[s];
  for (int s = k + 1; s < p->d; ++s) Rk *= p->n[s];
  const int64_t F = M * Rk;
  if (p->n[k] * F >= ((int64_t)1 << 31)) return hipErrorInvalidValue;   // fibre offsets carry a sign bit
  int modes[TT_MAX_ORDER];
  int nm = 0;
  for (int s = 1; s < p->d; ++s)
    if (s != k) modes[nm++] = s;
  uint32_t* keys = p->at<uint32_t>(p->o_fkeys);
  uint32_t* off = p->at<uint32_t>(p->o_cnt);
  int64_t nb = 0, chunk = 0;
  hipError_t e = sort_keys(p, modes, nm, F, keys, off, &nb, &chunk);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sort_place<true>, dim3((unsigned)nb), dim3(kSortThreads), sizeof(uint32_t) * p->J, p->stream,
                     keys, F, chunk, p->at<uint32_t>(p->o_hist), off, (int32_t)p->J, (uint32_t*)nullptr,
                     p->at<uint2>(p->o_fsort), (uint32_t)M, (uint32_t)(p->n[k] * M));
  return hipGetLastError();
}
