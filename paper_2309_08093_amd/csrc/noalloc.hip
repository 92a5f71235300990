// Relative residual without a plan or a workspace, for callers that cannot
// allocate device memory.  The residual pass of k_residual.hip keeps three
// scratch arrays: its per-wave partials, u(o) (one R_2-vector per outer tuple)
// and H = G_0 x G_1 (n_0 n_1 x R_2).  Here they live in one fixed device
// array per GPU instead of a caller workspace.
#include <math.h>

#include <mutex>

#include "tt_internal.h"

// The scratch of tt_residual_noalloc.  Each GPU the library runs on holds one
// copy for the life of the process.  Host code never uses this name as an
// address: the device address comes from hipGetSymbolAddress (noalloc_scratch).
static __device__ __align__(256) char scratch[TT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices];

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
tt_status noalloc_scratch(char** out) {
  int dev = 0;
  TT_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return tt_fail(TT_ERR_ARG, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    TT_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return tt_fail(TT_ERR_HIP, "hipGetSymbolAddress returned a null scratch address");
    g_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_ptr[dev];
  return TT_OK;
}

}  // namespace

tt_status tt_residual_noalloc(int32_t d, const int64_t* n, const int64_t* r, tt_dtype x_dtype, tt_dtype work_dtype,
                              const void* X, const void* const* cores, void* hip_stream, double* rel_residual) {
  if (!n || !r || !X || !cores || !rel_residual) return tt_fail(TT_ERR_ARG, "null argument");
  if (d < 2 || d > TT_MAX_ORDER) return tt_fail(TT_ERR_SHAPE, "order d=%d outside [2, %d]", d, TT_MAX_ORDER);
  if (x_dtype != TT_F64 && x_dtype != TT_F32 && x_dtype != TT_BF16) return tt_fail(TT_ERR_ARG, "bad x_dtype");
  if (work_dtype != TT_F64 && work_dtype != TT_F32) return tt_fail(TT_ERR_ARG, "work_dtype must be F64 or F32");
  if (r[0] != 1 || r[d] != 1) return tt_fail(TT_ERR_SHAPE, "boundary ranks must be 1");
  for (int k = 0; k < d; ++k)
    if (!cores[k]) return tt_fail(TT_ERR_ARG, "core %d is null", k);
  tt_plan_s p{};
  p.d = d;
  int64_t N = 1;
  for (int k = 0; k < d; ++k) {
    if (n[k] < 1 || n[k] > (int64_t)1 << 30) return tt_fail(TT_ERR_SHAPE, "n[%d]=%lld out of range", k, (long long)n[k]);
    if (N > ((int64_t)1 << 46) / n[k]) return tt_fail(TT_ERR_SHAPE, "tensor too large");
    N *= n[k];
    p.n[k] = n[k];
  }
  for (int k = 0; k <= d; ++k) {
    if (r[k] < 1 || r[k] > TT_MAX_RANK) return tt_fail(TT_ERR_SHAPE, "r[%d]=%lld outside [1, %d]", k, (long long)r[k], TT_MAX_RANK);
    p.r[k] = r[k];
  }
  p.N = N;
  p.O0 = N / (n[0] * n[1]);
  if (p.O0 >= ((int64_t)1 << 31)) return tt_fail(TT_ERR_SHAPE, "prod n[2..d-1] must be < 2^31");
  if (n[0] * n[1] >= ((int64_t)1 << 31)) return tt_fail(TT_ERR_SHAPE, "n[0] n[1] must be < 2^31");
  p.xdt = x_dtype;
  p.wdt = work_dtype;
  p.res_waves = tt_residual_waves(p.O0, n[1]);
  p.stream = static_cast<hipStream_t>(hip_stream);
  p.user_stream = p.stream;
  for (int k = 0; k < d; ++k) p.tab_off[k + 1] = p.tab_off[k] + n[k];
  // layout: partials (2 per wave, then the 3 results), u(o), and H when it fits
  const size_t ws = p.wsize();
  const size_t b_res = align256(sizeof(double) * (2 * p.res_waves + 8));
  const size_t b_u = align256(ws * (size_t)p.O0 * (size_t)r[2]);
  const size_t b_h = align256(ws * (size_t)(n[0] * n[1]) * (size_t)r[2]);
  if (b_res + b_u > (size_t)TT_NOALLOC_SCRATCH_BYTES)
    return tt_fail(TT_ERR_SHAPE, "residual scratch of %zu bytes (partials and u(o) of %lld outer tuples x R_2 = %lld) "
                   "exceeds TT_NOALLOC_SCRATCH_BYTES = %d", b_res + b_u, (long long)p.O0, (long long)r[2],
                   (int)TT_NOALLOC_SCRATCH_BYTES);
  p.o_res = 0;
  p.o_resU = b_res;
  p.o_resH = b_res + b_u + b_h <= (size_t)TT_NOALLOC_SCRATCH_BYTES ? b_res + b_u : 0;   // 0: rows formed per task
  char* base = nullptr;
  tt_status st = noalloc_scratch(&base);
  if (st) return st;
  p.ws = base;
  p.ws_bytes = TT_NOALLOC_SCRATCH_BYTES;
  p.ws_need = b_res + b_u + (p.o_resH ? b_h : 0);
  // every wave writes its partial and the two kernels before the pass write
  // all of u(o) and H, so nothing in the scratch needs clearing
  const CoreDesc cd = tt_make_desc(&p, cores);
  TT_HIP_TRY(launch_residual(&p, X, cd));
  double host[3];
  TT_HIP_TRY(hipMemcpyAsync(host, base + p.o_res + sizeof(double) * 2 * p.res_waves, sizeof host,
                            hipMemcpyDeviceToHost, p.stream));
  TT_HIP_TRY(hipStreamSynchronize(p.stream));
  *rel_residual = host[0];
  if (!isfinite(host[0])) return tt_fail(TT_ERR_NONFINITE, "residual is not finite (%g / %g)", host[1], host[2]);
  return TT_OK;
}
