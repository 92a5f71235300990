// Seeded TensorSketch tables, the derived per-fibre key tables, and the
// counting sorts of fibres and outer tuples by key that the data sketches
// read.
//
// Tables (Sec. 2.2, Definitions of CountSketch and TensorSketch; Algorithm 1
// draws new operators once per outer iteration): every entry of h_s and v_s
// is an independent SplitMix64 output (Steele, Lea, Flood 2014), generated
// directly on the device, one thread per entry.
#include <cstring>

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
__device__ __forceinline__ void gen_tables_body(uint32_t* tab, const TabArgs& a, int32_t g) {
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

__global__ void k_gen_tables(uint32_t* tab, TabArgs a) { gen_tables_body(tab, a, blockIdx.x * blockDim.x + threadIdx.x); }

// Batched: the tables of problem blockIdx.y (its arguments in device memory).
struct BTab {
  uint32_t* tab;
  TabArgs a;
};
__global__ void kb_gen_tables(const BTab* __restrict__ A) {
  const BTab& t = A[blockIdx.y];
  gen_tables_body(t.tab, t.a, blockIdx.x * blockDim.x + threadIdx.x);
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
// global atomics.  One launch set sorts several tuple sets at once (the
// outer tuples of the k = 0 sketch and the fibres of every key-grouped
// k >= 1 sketch of a sweep): each is a job, and the tuples of a job are cut
// into nb contiguous chunks.
//  1. k_sort_count: one workgroup per (job, chunk w) computes the keys of the
//     chunk, stores them, counts them per bucket in LDS and writes the
//     counts to hist[w][.] of its job.
//  2. k_sort_scan (one workgroup per job): per bucket b, hist[w][b] becomes
//     the number of earlier-chunk tuples in b; the bucket totals are scanned
//     into off[0..J] (off[J] = number of tuples).
//  3. k_sort_place: chunk w's tuples of bucket b go to positions
//     off[b] + hist[w][b] onward, ranked inside the chunk by LDS atomics.
// The order inside a bucket follows those atomics and is not fixed; the data
// sketches that read the lists sum in FP64, so their output does not show it.
constexpr int kSortThreads = 1024;
constexpr int kSortPerThread = 8;       // tuples per thread and round, loaded before they are used
constexpr int64_t kSortMaxChunks = 64;

struct SortJob {
  int64_t count, chunk;   // tuples, tuples per chunk
  int32_t nb, blk0;       // chunks, first workgroup of the count and place launches
  int32_t lo, ex;         // the tuple's modes: lo..d-1 except ex, the first varying fastest
  int32_t fibre;          // list entry layout: fibre (uint2) or outer tuple (uint32)
  uint32_t M, nkM;        // fibre t = mu + M rho -> offset rho nkM + mu
  uint32_t* keys;
  uint32_t* hist;         // nb x J
  uint32_t* off;          // J + 1
  void* list;
};

struct SortArgs {
  const uint32_t* tab;
  int32_t tab_off[TT_MAX_ORDER];
  int32_t n[TT_MAX_ORDER];
  int32_t d, njobs;
  uint32_t J;
  SortJob job[TT_MAX_ORDER];
};

// the job of workgroup b of a count / place launch (uniform across the workgroup)
__device__ __forceinline__ int job_of(const SortArgs& a, int b) {
  int j = 0;
  while (j + 1 < a.njobs && b >= a.job[j + 1].blk0) ++j;
  return j;
}

__device__ __forceinline__ uint32_t job_key(uint32_t q, const SortArgs& a, int lo, int ex) {
  uint32_t rem = q, key = 0;
  for (int s = lo; s < a.d; ++s) {
    if (s == ex) continue;
    const uint32_t ns = (uint32_t)a.n[s], nxt = rem / ns;
    key = key_add(key, a.tab[a.tab_off[s] + (rem - nxt * ns)], a.J);
    rem = nxt;
  }
  return key;
}

__device__ __forceinline__ void sort_count_body(const SortArgs& a, int j, int w) {
  extern __shared__ uint32_t h[];   // J
  const int64_t count = a.job[j].count, chunk = a.job[j].chunk;
  const int lo_mode = a.job[j].lo, ex = a.job[j].ex;
  uint32_t* __restrict__ keys = a.job[j].keys;
  for (uint32_t b = threadIdx.x; b < a.J; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  const int64_t lo = w * chunk, hi = lo + chunk < count ? lo + chunk : count;
  for (int64_t q0 = lo + threadIdx.x; q0 < hi; q0 += (int64_t)kSortPerThread * blockDim.x) {
    uint32_t key[kSortPerThread];
#pragma unroll
    for (int u = 0; u < kSortPerThread; ++u) {
      const int64_t q = q0 + (int64_t)u * blockDim.x;
      key[u] = q < hi ? job_key((uint32_t)q, a, lo_mode, ex) : 0u;
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
  uint32_t* out = a.job[j].hist + (int64_t)w * a.J;
  for (uint32_t b = threadIdx.x; b < a.J; b += blockDim.x) out[b] = h[b];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_count(SortArgs a) {
  const int j = job_of(a, blockIdx.x);
  sort_count_body(a, j, blockIdx.x - a.job[j].blk0);
}

// Batched: the argument sets of several plans in device memory, src[b] =
// (argument set, chunk) of workgroup b (job 0 of each set).
__global__ __launch_bounds__(kSortThreads) void kb_sort_count(const SortArgs* __restrict__ A,
                                                              const int2* __restrict__ src) {
  const int2 t = src[blockIdx.x];
  sort_count_body(A[t.x], 0, t.y);
}

__device__ __forceinline__ void sort_scan_body(const SortArgs& a, int j) {
  extern __shared__ uint32_t tot[];   // J
  __shared__ uint32_t wsum[kSortThreads / 64];
  const int J = (int)a.J, nb = a.job[j].nb;
  uint32_t* __restrict__ hist = a.job[j].hist;
  uint32_t* __restrict__ off = a.job[j].off;
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

__global__ __launch_bounds__(kSortThreads) void k_sort_scan(SortArgs a) { sort_scan_body(a, blockIdx.x); }

__global__ __launch_bounds__(kSortThreads) void kb_sort_scan(const SortArgs* __restrict__ A) {
  sort_scan_body(A[blockIdx.x], 0);
}

// Fibre lists (the k >= 1 sketch): tuple t = mu + M rho of a column (modes
// 1..k-1 give mu, modes k+1..d-1 give rho) stored as {column-independent
// fibre offset rho n_k M + mu with the key's sign bit; bucket}.  Outer lists
// (the k = 0 sketch): {t with the key's sign bit}.
__device__ __forceinline__ void sort_place_body(const SortArgs& a, int j, int w) {
  extern __shared__ uint32_t h[];   // J
  const int J = (int)a.J;
  const int64_t count = a.job[j].count, chunk = a.job[j].chunk;
  const uint32_t* __restrict__ keys = a.job[j].keys;
  const uint32_t* hw = a.job[j].hist + (int64_t)w * J;
  const uint32_t* off = a.job[j].off;
  const bool fibre = a.job[j].fibre != 0;
  const uint32_t M = a.job[j].M, nkM = a.job[j].nkM;
  uint32_t* __restrict__ sorted = static_cast<uint32_t*>(a.job[j].list);
  uint2* __restrict__ fsorted = static_cast<uint2*>(a.job[j].list);
  for (int b = threadIdx.x; b < J; b += blockDim.x) h[b] = off[b] + hw[b];
  __syncthreads();
  const int64_t lo = w * chunk, hi = lo + chunk < count ? lo + chunk : count;
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
        if (fibre) {
          const uint32_t rho = (uint32_t)q / M, mu = (uint32_t)q - rho * M;
          fsorted[pos] = make_uint2((rho * nkM + mu) | (key[u] & TT_KEY_SIGN), c);
        } else {
          sorted[pos] = (uint32_t)q | (key[u] & TT_KEY_SIGN);
        }
      }
    }
  }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_place(SortArgs a) {
  const int j = job_of(a, blockIdx.x);
  sort_place_body(a, j, blockIdx.x - a.job[j].blk0);
}

__global__ __launch_bounds__(kSortThreads) void kb_sort_place(const SortArgs* __restrict__ A,
                                                              const int2* __restrict__ src) {
  const int2 t = src[blockIdx.x];
  sort_place_body(A[t.x], 0, t.y);
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

// The batched generator's argument set of plan p (host memory, the sweep
// index read from the plan's device counter); launch over nprob sets with
// max_entries the largest table size.
size_t tt_tab_args_bytes() { return sizeof(BTab); }
hipError_t tt_tab_args(const tt_plan_s* p, void* out) {
  if (!p->dsweep) return hipErrorInvalidValue;
  BTab t{};
  t.tab = p->at<uint32_t>(p->o_tab);
  for (int s = 0; s <= p->d; ++s) t.a.off[s] = (int32_t)p->tab_off[s];
  t.a.d = p->d;
  t.a.J = (uint32_t)p->J;
  t.a.seed = p->seed;
  t.a.sweep = 0;
  t.a.dsweep = p->dsweep;
  std::memcpy(out, &t, sizeof t);
  return hipSuccess;
}
hipError_t launch_gen_tables_batched(const void* args, int32_t nprob, int64_t max_entries, hipStream_t st) {
  if (nprob <= 0 || max_entries <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_gen_tables, dim3(nblk(max_entries, 256), (unsigned)nprob), dim3(256), 0, st,
                     static_cast<const BTab*>(args));
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

// Job of sort slot `slot`: 0 = the outer tuples of the k = 0 sketch (modes
// 2..d-1), k >= 1 = the fibres of mode k (modes 1..d-1 except k).
hipError_t add_job(const tt_plan_s* p, int slot, SortArgs& a, int32_t& blocks) {
  SortJob& jb = a.job[a.njobs];
  int64_t count = 1;
  if (slot == 0) {
    count = p->O0;
    jb.lo = 2;
    jb.ex = -1;
    jb.fibre = 0;
    jb.M = jb.nkM = 1;
    jb.list = p->at<uint32_t>(p->o_sortO);
    jb.off = p->at<uint32_t>(p->o_cnt);
  } else {
    int64_t M = 1, Rk = 1;
    for (int s = 1; s < slot; ++s) M *= p->n[s];
    for (int s = slot + 1; s < p->d; ++s) Rk *= p->n[s];
    count = M * Rk;
    if (p->n[slot] * count >= ((int64_t)1 << 31)) return hipErrorInvalidValue;   // offsets carry a sign bit
    jb.lo = 1;
    jb.ex = slot;
    jb.fibre = 1;
    jb.M = (uint32_t)M;
    jb.nkM = (uint32_t)(p->n[slot] * M);
    jb.list = p->at<uint2>(p->o_flist) + p->flist_off[slot];
    jb.off = p->at<uint32_t>(p->o_foff) + (int64_t)slot * (p->J_cap + 1);
  }
  if (count < 1 || count >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  jb.count = count;
  jb.nb = (int32_t)tt_sort_chunks(count);
  jb.chunk = (count + jb.nb - 1) / jb.nb;
  jb.blk0 = blocks;
  jb.keys = p->at<uint32_t>(p->o_skeys) + p->skeys_off[slot];
  jb.hist = p->at<uint32_t>(p->o_hist) + p->hist_off[slot];
  blocks += jb.nb;
  a.njobs += 1;
  return hipSuccess;
}

hipError_t run_sorts(const tt_plan_s* p, const int* slots, int nslots) {
  if (nslots <= 0) return hipSuccess;
  SortArgs a{};
  a.tab = p->at<uint32_t>(p->o_tab);
  for (int s = 0; s < p->d; ++s) {
    a.tab_off[s] = (int32_t)p->tab_off[s];
    a.n[s] = (int32_t)p->n[s];
  }
  a.d = p->d;
  a.J = (uint32_t)p->J;
  int32_t blocks = 0;
  hipError_t e;
  for (int i = 0; i < nslots; ++i)
    if ((e = add_job(p, slots[i], a, blocks)) != hipSuccess) return e;
  const size_t lds = sizeof(uint32_t) * p->J;
  hipLaunchKernelGGL(k_sort_count, dim3((unsigned)blocks), dim3(kSortThreads), lds, p->stream, a);
  hipLaunchKernelGGL(k_sort_scan, dim3((unsigned)a.njobs), dim3(kSortThreads), lds, p->stream, a);
  hipLaunchKernelGGL(k_sort_place, dim3((unsigned)blocks), dim3(kSortThreads), lds, p->stream, a);
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
// 2..d-1) grouped by their partial hash (o_sortO, offsets in o_cnt).
hipError_t launch_outer_sort(const tt_plan_s* p) {
  const int slot = 0;
  return run_sorts(p, &slot, 1);
}

// Sort the fibres of a mode-k column (k >= 1) by their key over modes != 0, k
// (list at tt_fibre_list(p, k)).
hipError_t launch_fibre_sort(const tt_plan_s* p, int k) {
  if (k < 1 || k >= p->d) return hipErrorInvalidValue;
  return run_sorts(p, &k, 1);
}

size_t tt_sort_args_bytes() { return sizeof(SortArgs); }

// The argument set of plan p's outer sort (one job, its chunks first), in
// host memory, for the batched launches; *nb = its chunks.
hipError_t tt_sort_args_outer(const tt_plan_s* p, void* out, int32_t* nb) {
  SortArgs a{};
  a.tab = p->at<uint32_t>(p->o_tab);
  for (int s = 0; s < p->d; ++s) {
    a.tab_off[s] = (int32_t)p->tab_off[s];
    a.n[s] = (int32_t)p->n[s];
  }
  a.d = p->d;
  a.J = (uint32_t)p->J;
  int32_t blocks = 0;
  const hipError_t e = add_job(p, 0, a, blocks);
  if (e != hipSuccess) return e;
  std::memcpy(out, &a, sizeof a);
  *nb = blocks;
  return hipSuccess;
}

// The argument set of the sort of plan p's mode-k slabs (k >= 2): the
// n_0 x n_1 slabs of a mode-k column (modes 2..d-1 except k; t = mu + M rho,
// modes 2..k-1 giving mu) by their key over those modes, as {column-
// independent slab offset rho n_k M + mu with the key's sign bit; bucket} in
// the plan's mode-k list (which holds the larger mode-k fibre list of the
// single-plan path).  Host memory, for the batched launches; *nb = chunks.
hipError_t tt_sort_args_slabs(const tt_plan_s* p, int k, void* out, int32_t* nb) {
  if (k < 2 || k >= p->d) return hipErrorInvalidValue;
  SortArgs a{};
  a.tab = p->at<uint32_t>(p->o_tab);
  for (int s = 0; s < p->d; ++s) {
    a.tab_off[s] = (int32_t)p->tab_off[s];
    a.n[s] = (int32_t)p->n[s];
  }
  a.d = p->d;
  a.J = (uint32_t)p->J;
  SortJob& jb = a.job[0];
  int64_t M = 1, Rk = 1;
  for (int s = 2; s < k; ++s) M *= p->n[s];
  for (int s = k + 1; s < p->d; ++s) Rk *= p->n[s];
  const int64_t count = M * Rk;
  if (count < 1 || p->n[k] * count >= ((int64_t)1 << 31)) return hipErrorInvalidValue;   // offsets carry a sign bit
  jb.lo = 2;
  jb.ex = k;
  jb.fibre = 1;
  jb.M = (uint32_t)M;
  jb.nkM = (uint32_t)(p->n[k] * M);
  jb.list = p->at<uint2>(p->o_flist) + p->flist_off[k];
  jb.off = p->at<uint32_t>(p->o_foff) + (int64_t)k * (p->J_cap + 1);
  jb.count = count;
  jb.nb = (int32_t)tt_sort_chunks(count);
  jb.chunk = (count + jb.nb - 1) / jb.nb;
  jb.blk0 = 0;
  jb.keys = p->at<uint32_t>(p->o_skeys) + p->skeys_off[k];
  jb.hist = p->at<uint32_t>(p->o_hist) + p->hist_off[k];
  a.njobs = 1;
  std::memcpy(out, &a, sizeof a);
  *nb = jb.nb;
  return hipSuccess;
}

// The sorts of several plans in one launch set: args = nsets argument sets
// (device memory), src = (set, chunk) per workgroup, nblocks workgroups.
hipError_t launch_outer_sorts_batched(const void* args, const void* src, int32_t nsets, int32_t nblocks, int32_t J,
                                      hipStream_t st) {
  if (nsets <= 0) return hipSuccess;
  const SortArgs* A = static_cast<const SortArgs*>(args);
  const int2* S = static_cast<const int2*>(src);
  const size_t lds = sizeof(uint32_t) * J;
  hipLaunchKernelGGL(kb_sort_count, dim3((unsigned)nblocks), dim3(kSortThreads), lds, st, A, S);
  hipLaunchKernelGGL(kb_sort_scan, dim3((unsigned)nsets), dim3(kSortThreads), lds, st, A);
  hipLaunchKernelGGL(kb_sort_place, dim3((unsigned)nblocks), dim3(kSortThreads), lds, st, A, S);
  return hipGetLastError();
}

// Every list one sweep's data sketches read, in one launch set: the outer
// tuples and the fibres of each key-grouped mode.
hipError_t launch_sweep_sorts(const tt_plan_s* p) {
  int slots[TT_MAX_ORDER];
  int ns = 0;
  slots[ns++] = 0;
  for (int k = 1; k < p->d; ++k)
    if (tt_sketch_use_gs(p, k)) slots[ns++] = k;
  return run_sorts(p, slots, ns);
}

const uint2* tt_fibre_list(const tt_plan_s* p, int k) { return p->at<uint2>(p->o_flist) + p->flist_off[k]; }
