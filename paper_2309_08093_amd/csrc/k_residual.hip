// Relative residual ||X - [[G]]||_F / ||X||_F (objective (3.1), Sec. 3).
//
// X is streamed once as mode-0 fibres.  Work units are (outer tuple o =
// (i_2..i_{d-1}), block of 64 consecutive i_1); a wave takes units in turn.
// For a unit it forms u = G_2(:,i_2,:) ... G_{d-1}(:,i_{d-1},0) (length R_2,
// entry b in lane b), then lane l computes w(i_1) = G_1(:,i_1,:) u for
// i_1 = block start + l (R_1 values in registers).  Fibres are read with
// 16-byte loads by lane groups as in the data sketch; each group fetches its
// fibre's w by shuffles and reconstructs T(i_0) = G_0(0,i_0,:) w with G_0 rows
// held in registers.  Squares are summed per fibre in the work type and
// accumulated in FP64; per-wave partials are summed in a fixed order.
#include "tt_internal.h"

namespace {

template <typename WT>
__device__ __forceinline__ WT to_work(double v) { return (WT)v; }
template <typename WT>
__device__ __forceinline__ WT to_work(float v) { return (WT)v; }
template <typename WT>
__device__ __forceinline__ WT to_work(uint16_t v) { return (WT)__uint_as_float((uint32_t)v << 16); }

template <typename XT, int V>
struct Vec {
  XT e[V];
};
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

template <typename XT, typename WT, int V, int NJ, int U>
__global__ __launch_bounds__(256) void k_residual(const XT* __restrict__ X, CoreDesc cd, double* __restrict__ part,
                                                  int64_t O, int32_t lpf_log2) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int TW = gridDim.x * (blockDim.x >> 6);
  const int LPF = 1 << lpf_log2;
  const int G = 64 >> lpf_log2;
  const int g = lane >> lpf_log2;
  const int v = lane & (LPF - 1);
  const int d = cd.d;
  const int n0 = cd.n[0], n1 = cd.n[1];
  const int R1 = cd.r1[0], R2 = cd.r1[1];
  const double* G0 = cd.G[0];
  const double* G1 = cd.G[1];
  // G_0 rows of this lane's positions (registers when few, else cached loads)
  constexpr bool kReg = NJ * V * sizeof(WT) <= 32;
  constexpr int NR = kReg ? NJ : 1;
  WT g0[NR][V][TT_MAX_RANK];
#pragma unroll
  for (int j = 0; j < NR; ++j)
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int i0 = (v + LPF * j) * V + e;
#pragma unroll
      for (int a = 0; a < TT_MAX_RANK; ++a)
        g0[j][e][a] = (kReg && i0 < n0 && a < R1) ? (WT)G0[i0 + (int64_t)n0 * a] : (WT)0;
    }
  const int nblk1 = (n1 + 63) / 64;
  const int64_t units = O * nblk1;
  double sd = 0.0, sx = 0.0;
  for (int64_t unit = gw; unit < units; unit += TW) {
    const int64_t o = unit / nblk1;
    const int i1lo = (int)(unit - o * nblk1) * 64;
    // u over modes d-1 .. 2 (lane b holds u_b)
    double u = lane == 0 ? 1.0 : 0.0;
    int ru = 1;
    {
      int64_t idx[TT_MAX_ORDER];
      int64_t rem = o;
      for (int s = 2; s < d; ++s) {
        idx[s] = rem % cd.n[s];
        rem /= cd.n[s];
      }
      for (int s = d - 1; s >= 2; --s) {
        const int r0 = cd.r0[s], ns = cd.n[s];
        const double* Gs = cd.G[s];
        double nu = 0.0;
        for (int b = 0; b < ru; ++b) {
          const double ub = __shfl(u, b, 64);
          if (lane < r0) nu += Gs[lane + (int64_t)r0 * (idx[s] + (int64_t)ns * b)] * ub;
        }
        u = lane < r0 ? nu : 0.0;
        ru = r0;
      }
    }
    double ub[TT_MAX_RANK];
#pragma unroll
    for (int b = 0; b < TT_MAX_RANK; ++b) ub[b] = __shfl(u, b, 64);
    // w(i_1) for i_1 = i1lo + lane
    WT wl[TT_MAX_RANK];
    {
      const int i1 = i1lo + lane;
#pragma unroll
      for (int a = 0; a < TT_MAX_RANK; ++a) {
        double acc = 0.0;
        if (a < R1 && i1 < n1)
#pragma unroll
          for (int b = 0; b < TT_MAX_RANK; ++b)
            if (b < R2) acc += G1[a + (int64_t)R1 * (i1 + (int64_t)n1 * b)] * ub[b];
        wl[a] = (WT)acc;
      }
    }
    const int nb = (n1 - i1lo) < 64 ? (n1 - i1lo) : 64;
    const XT* Xo = X + ((int64_t)o * n1 + i1lo) * (int64_t)n0;
    for (int t = 0; t < nb; t += G * U) {
      Vec<XT, V> x[U][NJ];
      bool ok[U];
      int fi[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        fi[q] = t + q * G + g;
        ok[q] = fi[q] < nb;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int p = (v + LPF * j) * V;
          if (ok[q] && p < n0) x[q][j] = load_vec<XT, V>(Xo + (int64_t)fi[q] * n0 + p);
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        WT wv[TT_MAX_RANK];
#pragma unroll
        for (int a = 0; a < TT_MAX_RANK; ++a) wv[a] = a < R1 ? (WT)__shfl(wl[a], fi[q] & 63, 64) : (WT)0;
        WT sdf = (WT)0, sxf = (WT)0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int p = (v + LPF * j) * V;
          if (ok[q] && p < n0) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              WT tt = (WT)0;
#pragma unroll
              for (int a = 0; a < TT_MAX_RANK; ++a)
                if (a < R1) tt += (kReg ? g0[kReg ? j : 0][e][a] : (WT)G0[p + e + (int64_t)n0 * a]) * wv[a];
              const WT xv = to_work<WT>(x[q][j].e[e]);
              const WT df = xv - tt;
              sdf += df * df;
              sxf += xv * xv;
            }
          }
        }
        sd += (double)sdf;
        sx += (double)sxf;
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

int ilog2_ceil(int64_t x) {
  int l = 0;
  while (((int64_t)1 << l) < x) ++l;
  return l;
}

template <typename XT, typename WT, int V, int NJ>
hipError_t run(const tt_plan_s* p, const XT* X, const CoreDesc& cd, int lpf) {
  constexpr int U = NJ >= 4 ? 1 : 4 / NJ;
  const int nw = (int)p->res_waves;
  double* part = p->at<double>(p->o_res);
  hipLaunchKernelGGL((k_residual<XT, WT, V, NJ, U>), dim3((unsigned)(nw / 4)), dim3(256), 0, p->stream, X, cd, part,
                     p->O0, lpf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, p->stream, part, nw, part + 2 * nw);
  return hipGetLastError();
}

template <typename XT, typename WT, int V>
hipError_t dispatch_v(const tt_plan_s* p, const XT* X, const CoreDesc& cd) {
  const int64_t vecs = (p->n[0] + V - 1) / V;
  int lpf = 6, nj = 1;
  if (vecs <= 64) lpf = ilog2_ceil(vecs);
  else nj = 1 << ilog2_ceil((vecs + 63) / 64);
  switch (nj) {
    case 1: return run<XT, WT, V, 1>(p, X, cd, lpf);
    case 2: return run<XT, WT, V, 2>(p, X, cd, lpf);
    case 4: return run<XT, WT, V, 4>(p, X, cd, lpf);
    case 8: return run<XT, WT, V, 8>(p, X, cd, lpf);
    case 16: return run<XT, WT, V, 16>(p, X, cd, lpf);
    case 32: return run<XT, WT, V, 32>(p, X, cd, lpf);
    default: return run<XT, WT, V, 64>(p, X, cd, lpf);
  }
}

template <typename XT, typename WT>
hipError_t dispatch(const tt_plan_s* p, const void* Xv, const CoreDesc& cd) {
  const XT* X = static_cast<const XT*>(Xv);
  constexpr int VV = 16 / (int)sizeof(XT);
  const bool vec = (p->n[0] % VV) == 0 && ((uintptr_t)Xv % 16) == 0;
  return vec ? dispatch_v<XT, WT, VV>(p, X, cd) : dispatch_v<XT, WT, 1>(p, X, cd);
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
