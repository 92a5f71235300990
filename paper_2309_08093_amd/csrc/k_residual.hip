// Relative residual ||X - [[G]]||_F / ||X||_F (objective (3.1), Sec. 3).
//
// X is streamed once as mode-0 fibres.  Each wave owns a set of outer tuples
// o = (i_2..i_{d-1}); for each it forms u = G_2(:,i_2,:) ... G_{d-1}(:,i_{d-1},0)
// (length R_2, one entry per lane), then for every i_1 the vector
// w = G_1(:,i_1,:) u (length R_1), and reconstructs the fibre entries
// T(i_0) = G_0(0,i_0,:) w with G_0 rows held in registers.  Squares are
// accumulated in FP64; per-wave partials are summed in a fixed order.
#include "tt_internal.h"

namespace {

template <typename WT>
__device__ __forceinline__ WT to_work(double v) { return (WT)v; }
template <typename WT>
__device__ __forceinline__ WT to_work(float v) { return (WT)v; }
template <typename WT>
__device__ __forceinline__ WT to_work(uint16_t v) { return (WT)__uint_as_float((uint32_t)v << 16); }

template <typename XT, typename WT, int NJ>
__global__ __launch_bounds__(256) void k_residual(const XT* __restrict__ X, CoreDesc cd, double* __restrict__ part,
                                                  int64_t O) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int TW = gridDim.x * (blockDim.x >> 6);
  const int d = cd.d;
  const int n0 = cd.n[0], n1 = cd.n[1];
  const int R1 = cd.r1[0], R2 = cd.r1[1];
  const double* G0 = cd.G[0];
  const double* G1 = cd.G[1];
  // rows of G_0 for this lane's positions: in registers when few, else read
  // through the cache
  constexpr bool kRegRows = NJ <= 4;
  constexpr int NR = kRegRows ? NJ : 1;
  WT g0[NR][TT_MAX_RANK];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int i0 = lane + 64 * j;
#pragma unroll
    for (int a = 0; a < TT_MAX_RANK; ++a)
      g0[j][a] = (kRegRows && i0 < n0 && a < R1) ? (WT)G0[i0 + (int64_t)n0 * a] : (WT)0;
  }
  double sd = 0.0, sx = 0.0;
  for (int64_t o = gw; o < O; o += TW) {
    // u over modes d-1 .. 2 (lane a holds u_a)
    double u = lane == 0 ? 1.0 : 0.0;
    int ru = 1;   // current length of u (R_d = 1)
    {
      int64_t idx[TT_MAX_ORDER];
      int64_t rem = o;
      for (int s = 2; s < d; ++s) {
        idx[s] = rem % cd.n[s];
        rem /= cd.n[s];
      }
      for (int s = d - 1; s >= 2; --s) {
        const int r0 = cd.r0[s], ns = cd.n[s];
        const double* G = cd.G[s];
        double nu = 0.0;
        for (int b = 0; b < ru; ++b) {
          const double ub = __shfl(u, b, 64);
          if (lane < r0) nu += G[lane + (int64_t)r0 * (idx[s] + (int64_t)ns * b)] * ub;
        }
        u = lane < r0 ? nu : 0.0;
        ru = r0;
      }
    }
    double ub[TT_MAX_RANK];
#pragma unroll
    for (int b = 0; b < TT_MAX_RANK; ++b) ub[b] = __shfl(u, b, 64);
    for (int i1 = 0; i1 < n1; ++i1) {
      double wl = 0.0;
      if (lane < R1) {
#pragma unroll
        for (int b = 0; b < TT_MAX_RANK; ++b)
          if (b < R2) wl += G1[lane + (int64_t)R1 * (i1 + (int64_t)n1 * b)] * ub[b];
      }
      WT wv[TT_MAX_RANK];
#pragma unroll
      for (int a = 0; a < TT_MAX_RANK; ++a) wv[a] = (WT)__shfl(wl, a, 64);
      const XT* base = X + ((int64_t)o * n1 + i1) * (int64_t)n0;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int i0 = lane + 64 * j;
        if (i0 < n0) {
          const WT x = to_work<WT>(base[i0]);
          WT t = (WT)0;
#pragma unroll
          for (int a = 0; a < TT_MAX_RANK; ++a)
            if (a < R1) t += (kRegRows ? g0[kRegRows ? j : 0][a] : (WT)G0[i0 + (int64_t)n0 * a]) * wv[a];
          const double df = (double)x - (double)t;
          sd += df * df;
          sx += (double)x * (double)x;
        }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    sd += __shfl_xor(sd, off, 64);
    sx += __shfl_xor(sx, off, 64);
  }
  if (lane == 0) {
    part[2 * gw] = sd;
    part[2 * gw + 1] = sx;
  }
}

// out[0] = sqrt(sd / sx), out[1] = sd, out[2] = sx; fixed summation order.
__global__ void k_residual_final(const double* __restrict__ part, int32_t nw, double* __restrict__ out) {
  __shared__ double a[256], b[256];
  double sd = 0.0, sx = 0.0;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) {
    sd += part[2 * i];
    sx += part[2 * i + 1];
  }
  a[threadIdx.x] = sd;
  b[threadIdx.x] = sx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      a[threadIdx.x] += a[threadIdx.x + st];
      b[threadIdx.x] += b[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sqrt(a[0] / b[0]);
    out[1] = a[0];
    out[2] = b[0];
  }
}

template <typename XT, typename WT, int NJ>
hipError_t run(const tt_plan_s* p, const XT* X, const CoreDesc& cd) {
  const int nw = (int)p->res_waves;
  double* part = p->at<double>(p->o_res);
  hipLaunchKernelGGL((k_residual<XT, WT, NJ>), dim3((unsigned)(nw / 4)), dim3(256), 0, p->stream, X, cd, part, p->O0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, p->stream, part, nw, part + 2 * nw);
  return hipGetLastError();
}

template <typename XT, typename WT>
hipError_t dispatch(const tt_plan_s* p, const void* Xv, const CoreDesc& cd) {
  const XT* X = static_cast<const XT*>(Xv);
  const int64_t n0 = p->n[0];
  if (n0 <= 64) return run<XT, WT, 1>(p, X, cd);
  if (n0 <= 128) return run<XT, WT, 2>(p, X, cd);
  if (n0 <= 256) return run<XT, WT, 4>(p, X, cd);
  if (n0 <= 512) return run<XT, WT, 8>(p, X, cd);
  if (n0 <= 1024) return run<XT, WT, 16>(p, X, cd);
  if (n0 <= 2048) return run<XT, WT, 32>(p, X, cd);
  return run<XT, WT, 64>(p, X, cd);
}

}  // namespace

hipError_t launch_residual(const tt_plan_s* p, const void* X, const CoreDesc& cd) {
  if (p->wdt == TT_F64) {
    if (p->xdt == TT_F64) return dispatch<double, double>(p, X, cd);
    if (p->xdt == TT_F32) return dispatch<float, double>(p, X, cd);
    return dispatch<uint16_t, double>(p, X, cd);
  }
  if (p->xdt == TT_F64) return dispatch<double, float>(p, X, cd);
  if (p->xdt == TT_F32) return dispatch<float, float>(p, X, cd);
  return dispatch<uint16_t, float>(p, X, cd);
}
