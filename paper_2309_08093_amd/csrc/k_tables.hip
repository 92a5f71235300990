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

// out[q] = combined key (sum of hashes mod J, product of signs) of tuple q.
__global__ void k_build_keys(uint32_t* out, int64_t count, KeyArgs a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  int64_t rem = q;
  uint32_t key = 0;
  for (int t = 0; t < a.nm; ++t) {
    const int s = a.modes[t];
    const int64_t i = rem % a.n[s];
    rem /= a.n[s];
    key = key_add(key, a.tab[a.tab_off[s] + i], a.J);
  }
  out[q] = key;
}

__global__ void k_fill_u32(uint32_t* p, int64_t count, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void k_count(const uint32_t* keys, int64_t count, uint32_t* cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) atomicAdd(&cnt[keys[i] & TT_KEY_MASK], 1u);
}

// Exclusive scan of cnt[0..J) into off[0..J]; cursor[c] = off[c].  One block.
__global__ void k_scan(const uint32_t* cnt, uint32_t* off, uint32_t* cursor, int32_t J) {
  // exclusive prefix sum of cnt[0..J) into off (and cursor), off[J] = total;
  // per-thread runs, then an inclusive scan by shuffles within each wave and
  // over the wave totals
  __shared__ uint32_t wsum[16];
  const int t = threadIdx.x, T = blockDim.x, lane = t & 63, w = t >> 6, NW = T >> 6;
  const int per = (J + T - 1) / T;
  const int lo = min(J, t * per), hi = min(J, lo + per);
  uint32_t s = 0;
  for (int c = lo; c < hi; ++c) s += cnt[c];
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
  for (int c = lo; c < hi; ++c) {   // cnt may alias cursor: read before writing
    const uint32_t v = cnt[c];
    off[c] = acc;
    cursor[c] = acc;
    acc += v;
  }
}

// sorted[pos] = q | sign(q) << 31 grouped by bucket.
__global__ void k_scatter(const uint32_t* keys, int64_t count, uint32_t* cursor, uint32_t* sorted) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const uint32_t key = keys[q];
  const uint32_t pos = atomicAdd(&cursor[key & TT_KEY_MASK], 1u);
  sorted[pos] = (uint32_t)q | (key & TT_KEY_SIGN);
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

hipError_t launch_build_keys_modes(const tt_plan_s* p, uint32_t* out, int64_t count, const int* modes, int nm) {
  KeyArgs a{};
  a.tab = p->at<uint32_t>(p->o_tab);
  for (int s = 0; s < p->d; ++s) {
    a.tab_off[s] = (int32_t)p->tab_off[s];
    a.n[s] = (int32_t)p->n[s];
  }
  for (int t = 0; t < nm; ++t) a.modes[t] = modes[t];
  a.nm = nm;
  a.J = (uint32_t)p->J;
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_keys, dim3(nblk(count, 256)), dim3(256), 0, p->stream, out, count, a);
  return hipGetLastError();
}

hipError_t launch_build_keys(const tt_plan_s* p, uint32_t* out, int64_t count, int first, int last) {
  int modes[TT_MAX_ORDER];
  int nm = 0;
  for (int s = first; s <= last; ++s) modes[nm++] = s;
  return launch_build_keys_modes(p, out, count, modes, nm);
}

// Fibre list of the k >= 1 sketch: fibre t = mu + M rho of a column (modes
// 1..k-1 give mu, modes k+1..d-1 give rho) goes to its key's bucket as
// {column-independent fibre offset rho n_k M + mu, with the key's sign bit;
//  the key's bucket}.
__global__ void k_scatter_fibres(const uint32_t* __restrict__ keys, int64_t F, int64_t M, int64_t nkM,
                                 uint32_t* __restrict__ cursor, uint2* __restrict__ sorted) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= F) return;
  const uint32_t key = keys[t];
  const uint32_t c = key & TT_KEY_MASK;
  const uint32_t pos = atomicAdd(&cursor[c], 1u);
  const int64_t rho = t / M, mu = t - rho * M;
  sorted[pos] = make_uint2((uint32_t)(rho * nkM + mu) | (key & TT_KEY_SIGN), c);
}

// Bucket lists of the k = 0 data sketch: the outer mode tuples (modes
// 2..d-1) grouped by their partial hash.  Uses o_KO as key scratch.
hipError_t launch_outer_sort(const tt_plan_s* p) {
  const int64_t O = p->O0;
  uint32_t* keys = p->at<uint32_t>(p->o_KO);
  uint32_t* cnt = p->at<uint32_t>(p->o_cnt);          // J+1
  uint32_t* cursor = p->at<uint32_t>(p->o_cursor);    // J
  uint32_t* sorted = p->at<uint32_t>(p->o_sortO);     // O
  hipError_t e;
  if (p->d >= 3) {
    e = launch_build_keys(p, keys, O, 2, p->d - 1);
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, p->stream, keys, (int64_t)1, 0u);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  // counts accumulate in cursor; the scan turns them into the J+1 offsets in
  // cnt and resets cursor to the offsets for the scatter.
  hipLaunchKernelGGL(k_fill_u32, dim3(nblk(p->J, 256)), dim3(256), 0, p->stream, cursor, p->J, 0u);
  hipLaunchKernelGGL(k_count, dim3(nblk(O, 256)), dim3(256), 0, p->stream, keys, O, cursor);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, p->stream, cursor, cnt, cursor, (int32_t)p->J);
  hipLaunchKernelGGL(k_scatter, dim3(nblk(O, 256)), dim3(256), 0, p->stream, keys, O, cursor, sorted);
  return hipGetLastError();
}

// Sort the fibres of a mode-k column (k >= 1) by their key over modes != 0, k.
// Offsets of the J buckets go to o_cnt (J+1 entries), the list to o_fsort.
hipError_t launch_fibre_sort(const tt_plan_s* p, int k) {
  int64_t M = 1, Rk = 1;
  for (int s = 1; s < k; ++s) M *= p->n[s];
  for (int s = k + 1; s < p->d; ++s) Rk *= p->n[s];
  const int64_t F = M * Rk;
  int modes[TT_MAX_ORDER];
  int nm = 0;
  for (int s = 1; s < p->d; ++s)
    if (s != k) modes[nm++] = s;
  uint32_t* keys = p->at<uint32_t>(p->o_fkeys);
  uint32_t* off = p->at<uint32_t>(p->o_cnt);
  uint32_t* cursor = p->at<uint32_t>(p->o_cursor);
  hipError_t e;
  if (nm > 0) {
    if ((e = launch_build_keys_modes(p, keys, F, modes, nm)) != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, p->stream, keys, (int64_t)1, 0u);
  }
  hipLaunchKernelGGL(k_fill_u32, dim3(nblk(p->J, 256)), dim3(256), 0, p->stream, cursor, p->J, 0u);
  hipLaunchKernelGGL(k_count, dim3(nblk(F, 256)), dim3(256), 0, p->stream, keys, F, cursor);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, p->stream, cursor, off, cursor, (int32_t)p->J);
  hipLaunchKernelGGL(k_scatter_fibres, dim3(nblk(F, 256)), dim3(256), 0, p->stream, keys, F, M, p->n[k] * M, cursor,
                     p->at<uint2>(p->o_fsort));
  return hipGetLastError();
}
