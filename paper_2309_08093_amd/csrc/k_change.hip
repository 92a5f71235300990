// Relative change of the TT cores between two iterates, the accuracy measure
// the experiments of Sec. 5 stop on: max_k ||G_k^{(t+1)} - G_k^{(t)}||_F /
// ||G_k^{(t+1)}||_F.  One workgroup per core sums (new - old)^2 and new^2 in
// FP64 (wave shuffles, then LDS across the four waves); one thread then forms
// the d ratios and their maximum.  Non-finite ratios (a zero core, NaN input)
// propagate into the maximum so that the host can report them.
#include "tt_internal.h"

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_core_diff(CoreDesc prev, CoreDesc cur, double* __restrict__ sums) {
  const int k = blockIdx.x;
  const int64_t m = (int64_t)cur.r0[k] * cur.n[k] * cur.r1[k];
  const double* a = prev.G[k];
  const double* b = cur.G[k];
  double dd = 0.0, bb = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += kThreads) {
    const double bi = b[i], di = bi - a[i];
    dd = fma(di, di, dd);
    bb = fma(bi, bi, bb);
  }
  for (int off = 32; off > 0; off >>= 1) {
    dd += __shfl_down(dd, off);
    bb += __shfl_down(bb, off);
  }
  __shared__ double red[2][kThreads / 64];
  const int w = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) {
    red[0][w] = dd;
    red[1][w] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) {
      s0 += red[0][i];
      s1 += red[1][i];
    }
    sums[2 * k] = s0;
    sums[2 * k + 1] = s1;
  }
}

// out[0] = max_k sqrt(sums[2k]) / sqrt(sums[2k+1]); a NaN ratio wins
__global__ void k_core_change_max(const double* __restrict__ sums, int d, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double m = 0.0;
  for (int k = 0; k < d; ++k) {
    const double q = sqrt(sums[2 * k]) / sqrt(sums[2 * k + 1]);
    m = (q > m || q != q) && m == m ? q : m;
  }
  out[0] = m;
}

}  // namespace

// sums: 2 d doubles of scratch; out: one double (both device)
hipError_t launch_core_change(const tt_plan_s* p, const CoreDesc& prev, const CoreDesc& cur, double* sums,
                              double* out) {
  hipLaunchKernelGGL(k_core_diff, dim3(p->d), dim3(kThreads), 0, p->stream, prev, cur, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_core_change_max, dim3(1), dim3(64), 0, p->stream, sums, p->d, out);
  return hipGetLastError();
}
