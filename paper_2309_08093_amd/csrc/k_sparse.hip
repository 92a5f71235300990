// Data sketch of a sparse tensor in O(nnz) (the complexity remark after
// Theorem 3, Sec. 3: only the nonzeros of A enter S A_(k)^T).  Input is COO:
// coords[e d + s] = i_s of nonzero e (int32, device), vals[e] its value in the
// plan's storage type.  Nonzero e adds prod_{s != k} v_s(i_s) vals[e] to
// bucket (sum_{s != k} h_s(i_s)) mod J of column i_k, the same scatter as the
// dense sketch restricted to the stored entries (repeated coordinates add).
//
// One thread per nonzero reads its d coordinates and the packed tables (a
// few KB, cache resident), and adds into an FP64 accumulator in global
// memory with one atomic per output; the all-mode variant reads each nonzero
// once and scatters it into all d sketches.  A final kernel rounds the
// accumulators to the work type.  FP64 sums make the result independent of
// the order of the atomics up to FP64 rounding, below the work type's.
// Coordinates outside [0, n_s) are skipped and set bit 2 of the status word
// (reported by the next synchronising call), so bad input cannot address
// memory outside the outputs.
#include "tt_internal.h"

namespace {

template <typename XT>
__device__ __forceinline__ double val_f64(XT v) { return (double)v; }
template <>
__device__ __forceinline__ double val_f64<uint16_t>(uint16_t v) { return (double)__uint_as_float((uint32_t)v << 16); }

struct SparseArgs {
  int32_t n[TT_MAX_ORDER];
  int32_t tab_off[TT_MAX_ORDER];
  int64_t col_off[TT_MAX_ORDER];   // first accumulator entry of Y_k (J entries per column)
  int32_t d, k;                     // k < 0: every mode
  uint32_t J;
};

__global__ void k_fill_zero_f64(double* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

template <typename XT>
__global__ __launch_bounds__(256) void k_sketch_sparse(const int32_t* __restrict__ coords, const XT* __restrict__ vals,
                                                       int64_t nnz, const uint32_t* __restrict__ tab, SparseArgs a,
                                                       double* __restrict__ acc, int32_t* __restrict__ status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int d = a.d;
  int32_t idx[TT_MAX_ORDER];
  uint32_t key[TT_MAX_ORDER];
  bool ok = true;
  for (int s = 0; s < d; ++s) {
    const int32_t i = coords[e * d + s];
    ok = ok && i >= 0 && i < a.n[s];
    idx[s] = i;
  }
  if (!ok) {
    atomicOr(status, 4);
    return;
  }
  // sum of all modes' hashes and product of their signs; mode k's part is
  // taken out again below
  uint32_t hsum = 0, sgn = 0;
  for (int s = 0; s < d; ++s) {
    key[s] = tab[a.tab_off[s] + idx[s]];
    hsum += key[s] & TT_KEY_MASK;   // < d J <= 16 * 8192
    sgn ^= key[s] & TT_KEY_SIGN;
  }
  const double x = val_f64<XT>(vals[e]);
  const int k0 = a.k < 0 ? 0 : a.k, k1 = a.k < 0 ? d : a.k + 1;
  for (int k = k0; k < k1; ++k) {
    const uint32_t b = (hsum - (key[k] & TT_KEY_MASK)) % a.J;
    const bool neg = ((sgn ^ key[k]) & TT_KEY_SIGN) != 0;
    // hardware FP64 add (coarse-grained device memory)
    unsafeAtomicAdd(acc + a.col_off[k] + (int64_t)a.J * idx[k] + b, neg ? -x : x);
  }
}

template <typename WT>
__global__ void k_round_acc(const double* __restrict__ acc, WT* __restrict__ Y, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) Y[i] = (WT)acc[i];
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// k >= 0: Y_k (J x n_k); k < 0: every mode, Y_k at offset J (n_0 + ... + n_{k-1})
hipError_t launch_sketch_sparse(const tt_plan_s* p, int64_t nnz, const int32_t* coords, const void* vals, int k,
                                void* Y) {
  SparseArgs a{};
  a.d = p->d;
  a.k = k;
  a.J = (uint32_t)p->J;
  int64_t total = 0;
  for (int s = 0; s < p->d; ++s) {
    a.n[s] = (int32_t)p->n[s];
    a.tab_off[s] = (int32_t)p->tab_off[s];
    a.col_off[s] = k < 0 ? p->J * p->tab_off[s] : 0;
  }
  total = k < 0 ? p->J * p->tab_off[p->d] : p->J * p->n[k];
  double* acc = p->at<double>(p->o_spacc);
  hipLaunchKernelGGL(k_fill_zero_f64, dim3(nblk(total, 256)), dim3(256), 0, p->stream, acc, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nnz > 0) {
    const uint32_t* tab = p->at<uint32_t>(p->o_tab);
    int32_t* status = p->at<int32_t>(p->o_status);
    const dim3 grid(nblk(nnz, 256));
    if (p->xdt == TT_F64)
      hipLaunchKernelGGL(k_sketch_sparse<double>, grid, dim3(256), 0, p->stream, coords,
                         static_cast<const double*>(vals), nnz, tab, a, acc, status);
    else if (p->xdt == TT_F32)
      hipLaunchKernelGGL(k_sketch_sparse<float>, grid, dim3(256), 0, p->stream, coords,
                         static_cast<const float*>(vals), nnz, tab, a, acc, status);
    else
      hipLaunchKernelGGL(k_sketch_sparse<uint16_t>, grid, dim3(256), 0, p->stream, coords,
                         static_cast<const uint16_t*>(vals), nnz, tab, a, acc, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (p->wdt == TT_F64)
    hipLaunchKernelGGL(k_round_acc<double>, dim3(nblk(total, 256)), dim3(256), 0, p->stream, acc,
                       static_cast<double*>(Y), total);
  else
    hipLaunchKernelGGL(k_round_acc<float>, dim3(nblk(total, 256)), dim3(256), 0, p->stream, acc,
                       static_cast<float*>(Y), total);
  return hipGetLastError();
}
