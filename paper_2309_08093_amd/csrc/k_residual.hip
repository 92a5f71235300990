// Relative residual ||X - [[G]]||_F / ||X||_F (objective (lrtt), Sec. 3).
//
// Write an entry as X(i_0, i_1, o) with o = (i_2, ..., i_{d-1}).  Its TT value
// is sum_b H(i_0, i_1, b) u_b(o), where H = G_0 x G_1 contracted over their
// shared rank (n_0 n_1 x R_2) and u(o) = G_2(:, i_2, :) ... G_{d-1}(:, i_{d-1}, 0).
//  * k_res_u: one thread per outer tuple o computes u(o) (length R_2).
//  * k_res_slab: X is a sequence of slabs of S = n_0 n_1 contiguous entries,
//    one per o.  A wave task is (tile of 64 V consecutive slab positions, run
//    of consecutive o).  Lane l keeps H(p, :) for its V positions p in
//    registers and, for each o of the run, reads its V entries of slab o with
//    one vector load, forms T = H(p, :) u(o) (u is the same for the whole wave)
//    and accumulates (X - T)^2 and X^2.  Squares are summed per o in the work
//    type and accumulated in FP64; per-wave partials are summed in a fixed
//    order.  This avoids the cancellation of ||X||^2 - 2<X, T> + ||T||^2.
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

// U[o * R2 + b] = u_b(o): the product of the core slices of modes 2..d-1,
// taken right to left (mode 2 varies fastest in o).
template <typename WT>
__global__ void k_res_u(CoreDesc cd, WT* __restrict__ U, int64_t O) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= O) return;
  const int d = cd.d;
  int idx[TT_MAX_ORDER];
  int64_t rem = o;
  for (int s = 2; s < d; ++s) {
    idx[s] = (int)(rem % cd.n[s]);
    rem /= cd.n[s];
  }
  double v[TT_MAX_RANK];
#pragma unroll
  for (int a = 0; a < TT_MAX_RANK; ++a) v[a] = a == 0 ? 1.0 : 0.0;
  int rv = 1;   // length of v
  for (int s = d - 1; s >= 2; --s) {
    const int r0 = cd.r0[s], ns = cd.n[s];
    const double* Gs = cd.G[s];
    double nv[TT_MAX_RANK];
#pragma unroll
    for (int a = 0; a < TT_MAX_RANK; ++a) {
      double acc = 0.0;
      if (a < r0)
#pragma unroll
        for (int b = 0; b < TT_MAX_RANK; ++b)
          if (b < rv) acc += Gs[a + (int64_t)r0 * (idx[s] + (int64_t)ns * b)] * v[b];
      nv[a] = acc;
    }
#pragma unroll
    for (int a = 0; a < TT_MAX_RANK; ++a) v[a] = nv[a];
    rv = r0;
  }
#pragma unroll
  for (int b = 0; b < TT_MAX_RANK; ++b)
    if (b < rv) U[o * rv + b] = (WT)v[b];
}

// H[p * R2 + b] = sum_a G_0(0, i_0, a) G_1(a, i_1, b) for slab position
// p = i_0 + n_0 i_1.
template <typename WT>
__global__ void k_res_h(CoreDesc cd, WT* __restrict__ H) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n0 = cd.n[0], n1 = cd.n[1];
  if (p >= (int64_t)n0 * n1) return;
  const int R1 = cd.r1[0], R2 = cd.r1[1];
  const int i0 = (int)(p % n0), i1 = (int)(p / n0);
  const double* G0 = cd.G[0];
  const double* G1 = cd.G[1];
  for (int b = 0; b < R2; ++b) {
    double acc = 0.0;
    for (int a = 0; a < R1; ++a) acc += G0[i0 + (int64_t)n0 * a] * G1[a + (int64_t)R1 * (i1 + (int64_t)n1 * b)];
    H[p * R2 + b] = (WT)acc;
  }
}

// RB: bound on R_2 (registers per position).  Hb: H precomputed (k_res_h) or
// null, then each task forms its rows itself.
template <typename XT, typename WT, int V, int RB>
__global__ __launch_bounds__(256) void k_res_slab(const XT* __restrict__ X, CoreDesc cd, const WT* __restrict__ U,
                                                  const WT* __restrict__ Hb, double* __restrict__ part, int64_t O,
                                                  int32_t orun) {
  const int lane = threadIdx.x & 63;
  // wave-uniform, so that task, o and the u(o) loads stay scalar
  const int gw = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const int TW = gridDim.x * (blockDim.x >> 6);
  const int n0 = cd.n[0], n1 = cd.n[1];
  const int R1 = cd.r1[0], R2 = cd.r1[1];
  const int64_t S = (int64_t)n0 * n1;
  const double* G0 = cd.G[0];
  const double* G1 = cd.G[1];
  const int64_t tiles = (S + 64 * V - 1) / (64 * V);
  const int64_t runs = (O + orun - 1) / orun;
  const int64_t tasks = tiles * runs;
  double sd = 0.0, sx = 0.0;
  for (int64_t task = gw; task < tasks; task += TW) {
    const int64_t tile = task % tiles, run = task / tiles;
    const int64_t p0 = (tile * 64 + lane) * V;
    // H(p, :) for the lane's positions
    WT h[V][RB];
    if (Hb) {
#pragma unroll
      for (int e = 0; e < V; ++e)
#pragma unroll
        for (int b = 0; b < RB; ++b) h[e][b] = (p0 + e < S && b < R2) ? Hb[(p0 + e) * R2 + b] : (WT)0;
    } else {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int64_t p = p0 + e;
        const int i0 = (int)(p % n0), i1 = (int)(p / n0);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          double acc = 0.0;
          if (p < S && b < R2)
            for (int a = 0; a < R1; ++a)
              acc += G0[i0 + (int64_t)n0 * a] * G1[a + (int64_t)R1 * (i1 + (int64_t)n1 * b)];
          h[e][b] = (WT)acc;
        }
      }
    }
    const bool ok = p0 < S;
    const int64_t oa = run * orun, oe = (oa + orun) < O ? oa + orun : O;
    // UO slabs per batch; the loads of the next batch are issued before the
    // current one is used, so a wave always has loads in flight
    constexpr int UO = 4;
    auto issue = [&](Vec<XT, V> (&x)[UO], int64_t ob) {
#pragma unroll
      for (int q = 0; q < UO; ++q)
        if (ok && ob + q < oe) x[q] = load_vec<XT, V>(X + (ob + q) * S + p0);
    };
    auto consume = [&](const Vec<XT, V> (&x)[UO], int64_t ob) {
#pragma unroll
      for (int q = 0; q < UO; ++q) {
        if (ob + q >= oe) break;
        const int64_t o = ob + q;
        WT u[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) u[b] = b < R2 ? U[o * R2 + b] : (WT)0;
        WT sdf = (WT)0, sxf = (WT)0;
        if (ok) {
#pragma unroll
          for (int e = 0; e < V; ++e) {
            if (p0 + e < S) {
              WT t = (WT)0;
#pragma unroll
              for (int b = 0; b < RB; ++b) t += h[e][b] * u[b];
              const WT xv = to_work<WT>(x[q].e[e]);
              const WT df = xv - t;
              sdf += df * df;
              sxf += xv * xv;
            }
          }
        }
        sd += (double)sdf;
        sx += (double)sxf;
      }
    };
    Vec<XT, V> xa[UO], xb[UO];
    if (oa < oe) issue(xa, oa);
    for (int64_t ob = oa; ob < oe; ob += 2 * UO) {
      if (ob + UO < oe) issue(xb, ob + UO);
      consume(xa, ob);
      if (ob + UO >= oe) break;
      if (ob + 2 * UO < oe) issue(xa, ob + 2 * UO);
      consume(xb, ob + UO);
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

template <typename XT, typename WT, int V, int RB>
hipError_t run(const tt_plan_s* p, const XT* X, const CoreDesc& cd, const WT* U, const WT* H) {
  const int nw = (int)p->res_waves;
  double* part = p->at<double>(p->o_res);
  const int64_t S = p->n[0] * p->n[1];
  const int64_t tiles = (S + 64 * V - 1) / (64 * V);
  // runs of outer tuples: enough tasks for every wave, long enough to
  // amortise forming H
  int64_t orun = (tiles * p->O0) / (2 * (int64_t)nw);
  if (orun < 4) orun = 4;
  if (orun > 512) orun = 512;
  hipLaunchKernelGGL((k_res_slab<XT, WT, V, RB>), dim3((unsigned)(nw / 4)), dim3(256), 0, p->stream, X, cd, U, H,
                     part, p->O0, (int32_t)orun);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, p->stream, part, nw, part + 2 * p->res_waves);
  return hipGetLastError();
}

template <typename XT, typename WT, int V>
hipError_t dispatch_r(const tt_plan_s* p, const XT* X, const CoreDesc& cd, const WT* U, const WT* H) {
  const int64_t R2 = p->r[2];
  if (R2 <= 4) return run<XT, WT, V, 4>(p, X, cd, U, H);
  if (R2 <= 8) return run<XT, WT, V, 8>(p, X, cd, U, H);
  if (R2 <= 12) return run<XT, WT, V, 12>(p, X, cd, U, H);
  return run<XT, WT, V, 16>(p, X, cd, U, H);
}

template <typename XT, typename WT>
hipError_t dispatch(const tt_plan_s* p, const void* Xv, const CoreDesc& cd) {
  const XT* X = static_cast<const XT*>(Xv);
  WT* U = p->at<WT>(p->o_resU);
  hipLaunchKernelGGL(k_res_u<WT>, dim3((unsigned)((p->O0 + 255) / 256)), dim3(256), 0, p->stream, cd, U, p->O0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // H = G_0 x G_1 once, when the plan's buffer holds it
  const int64_t S = p->n[0] * p->n[1];
  WT* H = nullptr;
  if (p->o_resH) {
    H = p->at<WT>(p->o_resH);
    hipLaunchKernelGGL(k_res_h<WT>, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, p->stream, cd, H);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // 16-byte loads, 8-byte for BF16 (eight BF16 positions per lane would
  // hold 64 H values in registers and cost two waves of occupancy)
  constexpr int VV = sizeof(XT) == 2 ? 4 : 16 / (int)sizeof(XT);
  const bool vec = (S % VV) == 0 && ((uintptr_t)Xv % 16) == 0;
  return vec ? dispatch_r<XT, WT, VV>(p, X, cd, U, H) : dispatch_r<XT, WT, 1>(p, X, cd, U, H);
}

}  // namespace

// Waves of the residual pass: one work unit per (outer tuple, block of 64
// i_1), four waves per unit, at most 2048 units.
int64_t tt_residual_waves(int64_t O0, int64_t n1) {
  int64_t rb = (O0 * ((n1 + 63) / 64) + 3) / 4;
  if (rb > 2048) rb = 2048;
  if (rb < 1) rb = 1;
  return 4 * rb;
}

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
