// C ABI of the TT-TensorSketch library: plan, workspace layout, validation,
// and the orchestration of Algorithm 1 (Sec. 3) on one HIP stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "tt_internal.h"

namespace {
thread_local char g_err[512] = "";

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

CoreDesc make_desc(const tt_plan_s* p, const void* const* cores) {
  CoreDesc cd{};
  cd.d = p->d;
  int64_t off = 0;
  for (int i = 0; i < p->d; ++i) {
    cd.G[i] = cores ? static_cast<const double*>(cores[i]) : nullptr;
    cd.r0[i] = (int32_t)p->r[i];
    cd.n[i] = (int32_t)p->n[i];
    cd.r1[i] = (int32_t)p->r[i + 1];
    cd.tab_off[i] = (int32_t)p->tab_off[i];
    cd.chat_off[i] = off;
    off += p->r[i] * p->r[i + 1];
  }
  return cd;
}

tt_status check_plan(tt_plan p) {
  if (!p) return tt_fail(TT_ERR_ARG, "null plan");
  if (!p->ws) return tt_fail(TT_ERR_WORKSPACE, "no workspace bound (tt_plan_bind_workspace)");
  return TT_OK;
}

tt_status check_cores(tt_plan p, const void* const* cores) {
  if (!cores) return tt_fail(TT_ERR_ARG, "null core array");
  for (int i = 0; i < p->d; ++i)
    if (!cores[i]) return tt_fail(TT_ERR_ARG, "core %d is null", i);
  return TT_OK;
}

tt_status gen_tables(tt_plan p) {
  TTProfScope ps(p, TT_PROF_TABLES);
  TT_HIP_TRY(launch_gen_tables(p, p->sweep));
  if (p->tw_J != p->J) {   // roots of unity of the FFTs, once per J
    TT_HIP_TRY(launch_fill_twiddles(p));
    p->tw_J = p->J;
  }
  p->override_tables = false;
  return TT_OK;
}

// QR + absorb of Algorithm 1's inner loop, k < d-1.
tt_status left_orth(tt_plan p, double* const* G, int k) {
  const int64_t m = p->r[k] * p->n[k], r = p->r[k + 1];
  TTProfScope ps(p, TT_PROF_QR);
  TT_HIP_TRY(launch_qr_core(p, G[k], m, r, 1, m));
  TT_HIP_TRY(launch_absorb_left(p, G[k + 1], r, p->n[k + 1] * p->r[k + 2]));
  return TT_OK;
}

// One step of the right-to-left orthogonalisation, k >= 1.
tt_status right_orth(tt_plan p, double* const* G, int k) {
  const int64_t m = p->n[k] * p->r[k + 1], r = p->r[k];
  TTProfScope ps(p, TT_PROF_QR);
  TT_HIP_TRY(launch_qr_core(p, G[k], m, r, r, 1));
  TT_HIP_TRY(launch_absorb_right(p, G[k - 1], p->r[k - 1] * p->n[k - 1], r));
  return TT_OK;
}

}  // namespace

void tt_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

tt_status tt_fail(tt_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

// ---------------------------------------------------------------- pieces of one sweep

CoreDesc tt_make_desc(const tt_plan_s* p, const void* const* cores) { return make_desc(p, cores); }
tt_status tt_plan_check(tt_plan p) { return check_plan(p); }

// Right-to-left orthogonalisation of every core (Alg. 1 keeps the cores
// right-orthogonal before each left-to-right pass), then the transformed
// CountSketches of cores 1..d-1 (core 0 enters no interface sketch of k = 0
// and is transformed after its own update).
tt_status tt_sweep_begin(tt_plan p, double* const* G, const CoreDesc& cd) {
  tt_status st;
  for (int k = p->d - 1; k >= 1; --k)
    if ((st = right_orth(p, G, k))) return st;
  TTProfScope ps(p, TT_PROF_INTERFACE);
  TT_HIP_TRY(launch_core_fft(p, cd, 0, p->d - 1, 0));
  return TT_OK;
}

// Interface sketch SH_k (Theorems 1-2) into the plan's SH buffer.
tt_status tt_sweep_interface(tt_plan p, const CoreDesc& cd, int k) {
  TTProfScope ps(p, TT_PROF_INTERFACE);
  TT_HIP_TRY(launch_interface_from_chat(p, cd, k, p->ws + p->o_SH));
  return TT_OK;
}

// Core update k from SH_k and the data sketch Y: Gram / right-hand side, the
// proximal solve in place, and for k < d-1 QR + absorb and the new transform
// of core k.
tt_status tt_sweep_update(tt_plan p, double* const* G, const CoreDesc& cd, int k, const void* Y) {
  {
    TTProfScope ps(p, TT_PROF_GRAM);
    TT_HIP_TRY(launch_gram(p, k, p->ws + p->o_SH, Y));
  }
  {
    TTProfScope ps(p, TT_PROF_SOLVE);
    TT_HIP_TRY(launch_prox_from_gram(p, k, G[k], G[k]));
  }
  if (k < p->d - 1) {
    tt_status st;
    if ((st = left_orth(p, G, k))) return st;
    TTProfScope ps(p, TT_PROF_INTERFACE);
    TT_HIP_TRY(launch_core_fft(p, cd, k, k, -1));
  }
  return TT_OK;
}

// Advance the sweep index and draw the next sweep's tables (unless they are
// overridden).
tt_status tt_sweep_end(tt_plan p) {
  p->sweep += 1;
  if (!p->override_tables) return gen_tables(p);
  return TT_OK;
}

extern "C" {

const char* tt_last_error(void) { return g_err; }
const char* tt_version(void) { return "tt_sketch 0.1 gfx950"; }

tt_status tt_sketch_plan(const tt_plan_desc* desc, void* hip_stream, size_t* workspace_bytes, tt_plan* out) {
  if (!desc || !workspace_bytes || !out) return tt_fail(TT_ERR_ARG, "null argument");
  const int d = desc->d;
  if (d < 2 || d > TT_MAX_ORDER) return tt_fail(TT_ERR_SHAPE, "order d=%d outside [2, %d]", d, TT_MAX_ORDER);
  if (!desc->n || !desc->r) return tt_fail(TT_ERR_ARG, "null n or r");
  if (desc->flags & ~(TT_FLAG_SERIAL | TT_FLAG_FUSE | TT_FLAG_NO_FUSE | TT_FLAG_EXACT | TT_FLAG_INNER |
                      TT_FLAG_NO_INNER))
    return tt_fail(TT_ERR_ARG, "unknown flags");
  if ((desc->flags & TT_FLAG_INNER) && (desc->flags & TT_FLAG_NO_INNER))
    return tt_fail(TT_ERR_ARG, "TT_FLAG_INNER and TT_FLAG_NO_INNER together");
  if ((desc->flags & TT_FLAG_FUSE) && (desc->flags & TT_FLAG_NO_FUSE))
    return tt_fail(TT_ERR_ARG, "TT_FLAG_FUSE and TT_FLAG_NO_FUSE together");
  if (desc->x_dtype != TT_F64 && desc->x_dtype != TT_F32 && desc->x_dtype != TT_BF16)
    return tt_fail(TT_ERR_ARG, "bad x_dtype");
  if (desc->work_dtype != TT_F64 && desc->work_dtype != TT_F32) return tt_fail(TT_ERR_ARG, "work_dtype must be F64 or F32");
  if (desc->gram_mode != TT_GRAM_WORK && desc->gram_mode != TT_GRAM_BF16) return tt_fail(TT_ERR_ARG, "bad gram_mode");
  if (desc->gram_mode == TT_GRAM_BF16 && desc->work_dtype != TT_F32)
    return tt_fail(TT_ERR_ARG, "TT_GRAM_BF16 needs work_dtype F32");
  if (!(desc->lambda >= 0.0) || !isfinite(desc->lambda)) return tt_fail(TT_ERR_ARG, "lambda must be finite and >= 0");
  const int64_t Jmax = desc->work_dtype == TT_F64 ? TT_MAX_J / 2 : TT_MAX_J;
  if (desc->J < 1 || desc->J > Jmax) return tt_fail(TT_ERR_ARG, "J=%lld outside [1, %lld]", (long long)desc->J, (long long)Jmax);
  int rad[32], nrad = 0;
  if (!tt_factor_fft(desc->J, rad, &nrad)) return tt_fail(TT_ERR_ARG, "J=%lld has a prime factor > 7", (long long)desc->J);
  if (desc->r[0] != 1 || desc->r[d] != 1) return tt_fail(TT_ERR_SHAPE, "boundary ranks must be 1");
  int64_t N = 1;
  for (int k = 0; k < d; ++k) {
    const int64_t nk = desc->n[k];
    if (nk < 1 || nk > (int64_t)1 << 30) return tt_fail(TT_ERR_SHAPE, "n[%d]=%lld out of range", k, (long long)nk);
    if (N > ((int64_t)1 << 46) / nk) return tt_fail(TT_ERR_SHAPE, "tensor too large");
    N *= nk;
  }
  if (desc->n[0] > TT_MAX_N0) return tt_fail(TT_ERR_SHAPE, "n[0]=%lld > %d", (long long)desc->n[0], TT_MAX_N0);
  for (int k = 1; k < d; ++k) {
    const int64_t rk = desc->r[k];
    if (rk < 1 || rk > TT_MAX_RANK) return tt_fail(TT_ERR_SHAPE, "r[%d]=%lld outside [1, %d]", k, (long long)rk, TT_MAX_RANK);
    if (rk > desc->r[k - 1] * desc->n[k - 1] || rk > desc->n[k] * desc->r[k + 1])
      return tt_fail(TT_ERR_SHAPE, "rank r[%d]=%lld is infeasible", k, (long long)rk);
  }
  for (int k = 0; k < d; ++k)
    if (desc->r[k] * desc->r[k + 1] > TT_MAX_S)
      return tt_fail(TT_ERR_SHAPE, "r[%d] r[%d] > %d", k, k + 1, TT_MAX_S);

  tt_plan_s* p = new (std::nothrow) tt_plan_s();
  if (!p) return tt_fail(TT_ERR_ARG, "out of host memory");
  p->d = d;
  for (int k = 0; k < d; ++k) p->n[k] = desc->n[k];
  for (int k = 0; k <= d; ++k) p->r[k] = desc->r[k];
  p->J = desc->J;
  p->J_cap = desc->J;
  p->dsweep = nullptr;
  p->lambda = desc->lambda;
  p->lambda0 = desc->lambda;
  p->seed = desc->seed;
  p->xdt = desc->x_dtype;
  p->wdt = desc->work_dtype;
  p->gram_mode = desc->gram_mode;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->user_stream = p->stream;
  p->side = nullptr;
  p->chain = nullptr;
  p->reserved_cus = TT_DEFAULT_RESERVED_CUS;
  p->sketch_cus = 0;
  p->flags = desc->flags;
  p->sweep = 0;
  p->override_tables = false;
  p->N = N;
  p->fft_nrad = nrad;
  for (int i = 0; i < nrad; ++i) p->fft_radix[i] = rad[i];

  p->tab_off[0] = 0;
  p->max_n = 0;
  for (int k = 0; k < d; ++k) {
    p->tab_off[k + 1] = p->tab_off[k] + p->n[k];
    if (p->n[k] > p->max_n) p->max_n = p->n[k];
  }
  p->s_max = 0;
  p->r_max = 1;
  p->chat_cols = 0;
  p->qr_m = 1;
  for (int k = 0; k < d; ++k) {
    const int64_t s = p->r[k] * p->r[k + 1];
    if (s > p->s_max) p->s_max = s;
    if (p->r[k + 1] > p->r_max) p->r_max = p->r[k + 1];
    p->chat_cols += s;
    const int64_t m1 = p->r[k] * p->n[k], m2 = p->n[k] * p->r[k + 1];
    if (m1 > p->qr_m) p->qr_m = m1;
    if (m2 > p->qr_m) p->qr_m = m2;
  }
  p->O0 = 1;
  for (int s = 2; s < d; ++s) p->O0 *= p->n[s];
  if (p->O0 >= ((int64_t)1 << 31)) {
    delete p;
    return tt_fail(TT_ERR_SHAPE, "prod n[2..d-1] must be < 2^31");
  }
  p->max_M = 1;
  for (int s = 1; s < d - 1; ++s) p->max_M *= p->n[s];
  p->max_R = p->O0 > 1 ? p->O0 : 1;
  p->part_entries = 1;
  for (int k = 1; k < d; ++k) {
    // the largest grid a launch can use gives the most partials per column
    // (for every J up to J_cap, see tt_plan_set_sketch)
    const int64_t Ftot = N / p->n[0];
    const int64_t W = Ftot < TT_SKETCH_MAX_WG ? Ftot : TT_SKETCH_MAX_WG;
    const int64_t e = p->n[k] * tt_sketch_slots(p, k, W) * p->J;
    if (e > p->part_entries) p->part_entries = e;
  }
  // fused k = 0 pass writing the outer sketch (TT_FLAG_FUSE); its Y_1 stage
  // keeps n_1 x slices partials of J entries
  bool fuse = false;
  if (d >= 3 && !(p->flags & TT_FLAG_NO_FUSE)) {
    const double zo_bytes = (double)p->wsize() * (double)p->J_cap * (double)p->n[0] * (double)p->n[1];
    fuse = (p->flags & TT_FLAG_FUSE) || 2.0 * zo_bytes <= 0.5 * (double)N * (double)p->xsize();
  }
  if (fuse) {
    const int64_t e = p->n[1] * tt_outer_slices(p) * p->J_cap;
    if (e > p->part_entries) p->part_entries = e;
  }
  // inner sketch Z over modes 0..m-1 (TT_FLAG_INNER): the m with the fewest
  // bytes moved, own passes for the modes 2..m-1; its Y_k stages keep n_k x
  // slices partials of J entries.  The pass that writes Z adds every entry
  // by an LDS atomic, about 1.6e12 per second on this device: an entry costs
  // at least the time of 4 bytes of HBM (measured at 64^5 BF16: 0.68 ms for
  // the pass against 0.35 ms for a key-grouped pass over X).
  bool inner = false;
  p->inner_m = 0;
  p->inner_rows = p->inner_O = 0;
  if (d >= 4 && p->n[0] <= 1024 && !(p->flags & TT_FLAG_NO_INNER)) {
    const double x_bytes = (double)N * (double)p->xsize();
    double best = 0.0;
    int64_t rows = 1;
    for (int m = 2; m <= d - 2; ++m) {
      rows *= p->n[m - 1];
      int64_t Om = 1;
      for (int s2 = m; s2 < d; ++s2) Om *= p->n[s2];
      // the slab's row keys and the J buckets fit in LDS
      if (rows > 16384) break;
      const double zi_bytes = (double)p->wsize() * (double)p->J_cap * (double)Om;
      const double pass = x_bytes > 4.0 * (double)N ? x_bytes : 4.0 * (double)N;
      const double bytes = (m - 2) * x_bytes + pass + (d - m + 1) * zi_bytes;
      if (p->inner_m == 0 || bytes < best) {
        best = bytes;
        p->inner_m = m;
        p->inner_rows = rows;
        p->inner_O = Om;
      }
    }
    inner = p->inner_m > 0 && ((p->flags & TT_FLAG_INNER) || best <= 0.75 * (d - 2) * x_bytes);
    if (!inner) p->inner_m = 0;
  }
  p->o_zi = 0;
  if (inner) {
    for (int k = p->inner_m; k < d; ++k) {
      const int64_t e = p->n[k] * tt_inner_slices(p, k) * p->J_cap;
      if (e > p->part_entries) p->part_entries = e;
    }
  }
  p->gram_chunks = tt_gram_chunks(p->J);
  // residual work units: (outer tuple, block of 64 i_1), four waves per block
  p->res_waves = tt_residual_waves(p->O0, p->n[1]);

  const size_t ws = p->wsize();
  const size_t gs = (p->gram_mode == TT_GRAM_BF16) ? 4 : 8;   // Gram partials: FP64 unless BF16 MFMA
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + (bytes ? bytes : 1));
    return at;
  };
  p->o_tab = take(sizeof(uint32_t) * p->tab_off[d]);
  p->o_KI = take(sizeof(uint32_t) * p->max_M);
  p->o_KO = take(sizeof(uint32_t) * p->max_R);
  p->o_cnt = take(sizeof(uint32_t) * (p->J + 1));
  p->o_sortO = take(sizeof(uint32_t) * p->max_R);
  p->o_part = take(sizeof(double) * p->part_entries);
  p->o_chat = take(2 * ws * p->J * p->chat_cols);
  p->o_pre = take(2 * ws * p->J * TT_MAX_RANK);
  p->o_suf = take(2 * ws * p->J * TT_MAX_RANK);
  p->o_tw = take(2 * ws * p->J);
  p->tw_J = 0;
  p->o_SH = take(ws * p->J * p->s_max);
  p->o_Y = take(ws * p->J * p->max_n);
  p->o_gram = take(gs * p->gram_chunks * p->s_max * (p->s_max + p->max_n));
  p->o_minv = take(sizeof(double) * tt_chol_out_doubles(p->s_max));   // L and its diagonal-block inverses
  p->o_gsum = take(sizeof(double) * p->s_max * (p->s_max + p->max_n));
  p->o_W = take(sizeof(double));
  p->o_qrA = take(sizeof(double) * p->qr_m * p->r_max);
  p->o_qrQ = take(sizeof(double) * p->qr_m * p->r_max);
  p->o_qrR = take(sizeof(double) * p->r_max * p->r_max);
  p->o_status = take(64);
  p->o_res = take(sizeof(double) * (2 * p->res_waves + 8));
  p->o_chg = take(sizeof(double) * (2 * TT_MAX_ORDER + 8));
  p->o_resU = take(ws * p->O0 * p->r[2]);   // u(o) of the residual, O0 x R_2
  // G_0 x G_1 of the residual (n_0 n_1 x R_2), when it is at most 2^26 entries
  const int64_t nH = p->n[0] * p->n[1] * p->r[2];
  p->o_resH = nH <= ((int64_t)1 << 26) ? take(ws * nH) : 0;
  p->o_gold = take(sizeof(double));
  p->o_Yall = take(ws * p->J * p->tab_off[d]);   // Y_k of every mode for one sweep
  // key sorts: slot 0 = the outer tuples (O0), slot k = the fibres of one
  // column of mode k (N / (n_0 n_k))
  {
    int64_t nkeys = 0, nlist = 0, nhist = 0;
    for (int s = 0; s < d; ++s) {
      const int64_t cnt = s == 0 ? p->O0 : N / (p->n[0] * p->n[s]);
      p->skeys_off[s] = nkeys;
      p->hist_off[s] = nhist;
      nkeys += cnt;
      nhist += p->J * tt_sort_chunks(cnt);
      p->flist_off[s] = nlist;
      if (s > 0) nlist += cnt;
    }
    p->o_skeys = take(sizeof(uint32_t) * nkeys);
    p->o_hist = take(sizeof(uint32_t) * nhist);
    p->o_flist = take(8 * (nlist > 0 ? nlist : 1));
    p->o_foff = take(sizeof(uint32_t) * d * (p->J + 1));
  }
  p->o_pol = take(sizeof(float) * TT_MAX_ORDER * (TT_JPOLICY_FEATURES + TT_JPOLICY_OUTPUTS));
  // outer sketch of the fused k = 0 pass (J_cap x n_0 x n_1)
  p->o_zo = fuse ? take(ws * (size_t)p->J_cap * (size_t)p->n[0] * (size_t)p->n[1]) : 0;
  // inner sketch of the pass of mode inner_m (J_cap x inner_O)
  p->o_zi = inner ? take(ws * (size_t)p->J_cap * (size_t)p->inner_O) : 0;
  p->o_zperm = inner ? take(sizeof(uint32_t) * (size_t)p->J_cap) : 0;
  p->o_spacc = take(sizeof(double) * (size_t)p->J_cap * (size_t)p->tab_off[d]);
  // exact update
  p->o_exphi = p->o_exch = p->o_expart = p->o_exgram = p->o_exmerge = 0;
  p->ex_phi = p->ex_chain = p->ex_part = 0;
  if (p->flags & TT_FLAG_EXACT) {
    tt_exact_sizes(p, &p->ex_phi, &p->ex_chain);
    const int64_t big = p->ex_phi > p->ex_chain ? p->ex_phi : p->ex_chain;
    p->ex_part = 8 * big < ((int64_t)1 << 22) ? (8 * big > 4096 ? 8 * big : 4096) : ((int64_t)1 << 22);
    p->o_exphi = take(ws * 2 * (size_t)p->ex_phi);
    p->o_exch = take(ws * 2 * (size_t)p->ex_chain);
    p->o_expart = take(sizeof(double) * (size_t)p->ex_part);
    p->o_exgram = take(sizeof(double) * 512);
    const int64_t nmerge = tt_exact_merge_doubles(p);
    p->o_exmerge = nmerge > 0 ? take(sizeof(double) * (size_t)nmerge) : 0;
  }
  p->ws_need = o;
  p->ws = nullptr;
  p->ws_bytes = 0;
  *workspace_bytes = o;
  *out = p;
  g_err[0] = 0;
  return TT_OK;
}

tt_status tt_plan_bind_workspace(tt_plan p, void* dev_ws, size_t bytes) {
  if (!p || !dev_ws) return tt_fail(TT_ERR_ARG, "null argument");
  if (bytes < p->ws_need) return tt_fail(TT_ERR_WORKSPACE, "workspace %zu bytes < required %zu", bytes, p->ws_need);
  if (((uintptr_t)dev_ws & 255) != 0) return tt_fail(TT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  p->ws = static_cast<char*>(dev_ws);
  p->ws_bytes = bytes;
  p->tw_J = 0;
  TT_HIP_TRY(hipMemsetAsync(p->ws + p->o_status, 0, 64, p->stream));
  return gen_tables(p);
}

tt_status tt_plan_set_stream(tt_plan p, void* s) {
  if (!p) return tt_fail(TT_ERR_ARG, "null plan");
  p->stream = static_cast<hipStream_t>(s);
  p->user_stream = p->stream;
  return TT_OK;
}

namespace {

void free_streams(tt_plan p) {
  if (!p->side) return;
  (void)hipStreamSynchronize(p->side);
  (void)hipStreamSynchronize(p->chain);
  (void)hipStreamDestroy(p->side);
  (void)hipStreamDestroy(p->chain);
  (void)hipEventDestroy(p->ev_fork);
  (void)hipEventDestroy(p->ev_join);
  (void)hipEventDestroy(p->ev_done);
  for (int k = 0; k < TT_MAX_ORDER; ++k) (void)hipEventDestroy(p->ev_y[k]);
  p->side = p->chain = nullptr;
}

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return n;
}

// CUs kept from the side stream: the plan's setting, or by default those of
// one XCD.  The runtime numbers CUs XCD by XCD (ncu / 8 per XCD), and a
// reservation of exactly one XCD keeps the two streams on separate L2s:
// measured on the 200^4 sweep with a pass over X per mode, 32 CUs gave
// 4.56 ms, 0 gave 4.94 ms, and 24, 40 or 48 (an XCD split between the
// streams) 5.46-5.63 ms.  When the k = 0 pass writes both intermediates
// (one pass over X per sweep) the core updates cannot start before it ends,
// and the short stages after it leave CUs free: there the default keeps no
// CU back (200^4: 3.04 ms against 3.41 ms with 32 and 3.40 ms with 16).
int reserved_of(const tt_plan_s* p, int ncu) {
  if (p->reserved_cus >= 0) return p->reserved_cus;
  if (tt_sketch_joint(p)) return 0;
  return (ncu >= 64 && ncu % 8 == 0) ? ncu / 8 : 0;
}

// The side stream carries the data sketches; its CU mask leaves the first
// reserved CUs (in the runtime's CU numbering) to the chain stream, so
// the short latency-bound kernels of the core updates are not queued behind
// the persistent sketch grids.
tt_status make_streams(tt_plan p) {
  if (p->side) return TT_OK;
  const int ncu = device_cus();
  const int reserved = reserved_of(p, ncu);
  if (reserved > 0 && ncu > reserved) {
    std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
    for (int i = reserved; i < ncu; ++i) mask[i / 32] |= 1u << (i % 32);
    TT_HIP_TRY(hipExtStreamCreateWithCUMask(&p->side, (uint32_t)mask.size(), mask.data()));
  } else {
    TT_HIP_TRY(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
  }
  TT_HIP_TRY(hipStreamCreateWithFlags(&p->chain, hipStreamNonBlocking));
  TT_HIP_TRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
  TT_HIP_TRY(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
  TT_HIP_TRY(hipEventCreateWithFlags(&p->ev_done, hipEventDisableTiming));
  for (int k = 0; k < TT_MAX_ORDER; ++k) TT_HIP_TRY(hipEventCreateWithFlags(&p->ev_y[k], hipEventDisableTiming));
  return TT_OK;
}

// restores the plan's launch stream when an overlapped sweep returns
struct StreamRestore {
  tt_plan p;
  ~StreamRestore() {
    p->stream = p->user_stream;
    p->sketch_cus = 0;
  }
};

}  // namespace

tt_status tt_plan_set_overlap(tt_plan p, int32_t reserved_cus) {
  if (!p) return tt_fail(TT_ERR_ARG, "null plan");
  const int ncu = device_cus();
  if (reserved_cus < 0 || (ncu > 0 && reserved_cus >= ncu))
    return tt_fail(TT_ERR_ARG, "reserved_cus=%d outside [0, %d)", reserved_cus, ncu);
  free_streams(p);
  p->reserved_cus = reserved_cus;
  return TT_OK;
}

tt_status tt_plan_destroy(tt_plan p) {
  if (p) {
    tt_prof_free(p);
    free_streams(p);
  }
  delete p;
  return TT_OK;
}

tt_status tt_plan_set_sweep(tt_plan p, int64_t t) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (t < 0) return tt_fail(TT_ERR_ARG, "sweep index must be >= 0");
  p->sweep = t;
  return gen_tables(p);
}

tt_status tt_plan_set_sketch(tt_plan p, int64_t J, double lambda) {
  if (!p) return tt_fail(TT_ERR_ARG, "null plan");
  if (J < 1 || J > p->J_cap) return tt_fail(TT_ERR_ARG, "J=%lld outside [1, %lld]", (long long)J, (long long)p->J_cap);
  int rad[32], nrad = 0;
  if (!tt_factor_fft(J, rad, &nrad)) return tt_fail(TT_ERR_ARG, "J=%lld has a prime factor > 7", (long long)J);
  if (!(lambda >= 0.0) || !isfinite(lambda)) return tt_fail(TT_ERR_ARG, "lambda must be finite and >= 0");
  p->J = J;
  p->lambda = lambda;
  p->fft_nrad = nrad;
  for (int i = 0; i < nrad; ++i) p->fft_radix[i] = rad[i];
  p->override_tables = false;
  if (p->ws) return gen_tables(p);
  return TT_OK;
}

tt_status tt_plan_get_sketch(tt_plan p, int64_t* J, double* lambda) {
  if (!p || !J || !lambda) return tt_fail(TT_ERR_ARG, "null argument");
  *J = p->J;
  *lambda = p->lambda;
  return TT_OK;
}

tt_status tt_plan_get_sweep(tt_plan p, int64_t* t) {
  if (!p || !t) return tt_fail(TT_ERR_ARG, "null argument");
  *t = p->sweep;
  return TT_OK;
}

tt_status tt_plan_get_tables(tt_plan p, int32_t s, int32_t* h, int8_t* v) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (s < 0 || s >= p->d || !h || !v) return tt_fail(TT_ERR_ARG, "bad mode or null output");
  const int64_t ns = p->n[s];
  std::vector<uint32_t> buf(ns);
  TT_HIP_TRY(hipMemcpyAsync(buf.data(), p->ws + p->o_tab + sizeof(uint32_t) * p->tab_off[s], sizeof(uint32_t) * ns,
                            hipMemcpyDeviceToHost, p->stream));
  TT_HIP_TRY(hipStreamSynchronize(p->stream));
  for (int64_t i = 0; i < ns; ++i) {
    h[i] = (int32_t)(buf[i] & TT_KEY_MASK);
    v[i] = (buf[i] & TT_KEY_SIGN) ? -1 : 1;
  }
  return TT_OK;
}

tt_status tt_plan_set_tables(tt_plan p, int32_t s, const int32_t* h, const int8_t* v) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (s < 0 || s >= p->d || !h || !v) return tt_fail(TT_ERR_ARG, "bad mode or null input");
  const int64_t ns = p->n[s];
  std::vector<uint32_t> buf(ns);
  for (int64_t i = 0; i < ns; ++i) {
    if (h[i] < 0 || h[i] >= p->J || (v[i] != 1 && v[i] != -1))
      return tt_fail(TT_ERR_ARG, "table entry %lld of mode %d out of range", (long long)i, s);
    buf[i] = (uint32_t)h[i] | (v[i] < 0 ? TT_KEY_SIGN : 0u);
  }
  TT_HIP_TRY(hipMemcpyAsync(p->ws + p->o_tab + sizeof(uint32_t) * p->tab_off[s], buf.data(), sizeof(uint32_t) * ns,
                            hipMemcpyHostToDevice, p->stream));
  TT_HIP_TRY(hipStreamSynchronize(p->stream));
  p->override_tables = true;
  return TT_OK;
}

tt_status tt_plan_sketch_path(tt_plan p, int32_t k, int32_t* path) {
  if (!p || !path) return tt_fail(TT_ERR_ARG, "null argument");
  if (k < 0 || k >= p->d) return tt_fail(TT_ERR_ARG, "k=%d out of range", k);
  *path = k == 0 ? TT_SKETCH_PATH_BUCKET : (tt_sketch_use_gs(p, k) ? TT_SKETCH_PATH_GROUPED : TT_SKETCH_PATH_STREAM);
  return TT_OK;
}

tt_status tt_sketch_tensor(tt_plan p, const void* X, int32_t k, void* Y) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (!X || !Y) return tt_fail(TT_ERR_ARG, "null X or Y");
  if (k < 0 || k >= p->d) return tt_fail(TT_ERR_ARG, "k=%d out of range", k);
  TT_HIP_TRY(launch_sketch_tensor(p, X, k, Y));
  return TT_OK;
}

tt_status tt_sketch_tensor_all(tt_plan p, const void* X, void* Yall) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (!X || !Yall) return tt_fail(TT_ERR_ARG, "null argument");
  struct ListsReady {
    tt_plan p;
    ~ListsReady() { p->lists_ready = false; }
  } lists_guard{p};
  {
    TTProfScope ps(p, TT_PROF_SKETCH_AUX);
    TT_HIP_TRY(launch_sweep_sorts(p));
  }
  p->lists_ready = true;
  const bool fused = tt_sketch_fused01(p);
  const bool inner = tt_sketch_inner(p);
  char* Yb = static_cast<char*>(Yall);
  for (int k = 0; k < p->d; ++k) {
    void* Yk = Yb + p->wsize() * p->J * p->tab_off[k];
    if (fused && k == 0) {
      TT_HIP_TRY(launch_sketch_mode0_outer(p, X, Yk));
    } else if (fused && k == 1) {
      TT_HIP_TRY(launch_sketch_y1_outer(p, Yk));
    } else if (inner && k >= p->inner_m) {
      if (k == p->inner_m) TT_HIP_TRY(launch_sketch_inner(p, X, Yall));
    } else {
      TT_HIP_TRY(launch_sketch_tensor(p, X, k, Yk));
    }
  }
  return TT_OK;
}

tt_status tt_sketch_sparse(tt_plan p, int64_t nnz, const int32_t* coords, const void* vals, int32_t k, void* Y) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (nnz < 0 || (nnz > 0 && (!coords || !vals)) || !Y) return tt_fail(TT_ERR_ARG, "null argument or nnz < 0");
  if (k < 0 || k >= p->d) return tt_fail(TT_ERR_ARG, "k=%d out of range", k);
  TTProfScope ps(p, TT_PROF_SKETCHK);
  TT_HIP_TRY(launch_sketch_sparse(p, nnz, coords, vals, k, Y));
  return TT_OK;
}

tt_status tt_sketch_sparse_all(tt_plan p, int64_t nnz, const int32_t* coords, const void* vals, void* Yall) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (nnz < 0 || (nnz > 0 && (!coords || !vals)) || !Yall) return tt_fail(TT_ERR_ARG, "null argument or nnz < 0");
  TTProfScope ps(p, TT_PROF_SKETCHK);
  TT_HIP_TRY(launch_sketch_sparse(p, nnz, coords, vals, -1, Yall));
  return TT_OK;
}

tt_status tt_plan_sketch_sources(tt_plan p, int32_t* src) {
  if (!p || !src) return tt_fail(TT_ERR_ARG, "null argument");
  for (int k = 0; k < p->d; ++k) src[k] = k;
  if (tt_sketch_fused01(p)) src[1] = 0;
  if (tt_sketch_inner(p))
    for (int k = p->inner_m + 1; k < p->d; ++k) src[k] = p->inner_m;
  if (tt_sketch_joint(p))
    for (int k = 2; k < p->d; ++k) src[k] = 0;
  return TT_OK;
}

tt_status tt_sketch_interface(tt_plan p, const void* const* cores, int32_t k, void* SH) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (k < 0 || k >= p->d) return tt_fail(TT_ERR_ARG, "k=%d out of range", k);
  if (!cores || !SH) return tt_fail(TT_ERR_ARG, "null argument");
  for (int i = 0; i < p->d; ++i)
    if (i != k && !cores[i]) return tt_fail(TT_ERR_ARG, "core %d is null", i);
  const CoreDesc cd = make_desc(p, cores);
  TTProfScope ps(p, TT_PROF_INTERFACE);
  TT_HIP_TRY(launch_core_fft(p, cd, 0, p->d - 1, k));
  TT_HIP_TRY(launch_interface_from_chat(p, cd, k, SH));
  return TT_OK;
}

tt_status tt_prox_solve(tt_plan p, int32_t k, const void* SH, const void* Y, const void* G_old, void* G_new) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (k < 0 || k >= p->d) return tt_fail(TT_ERR_ARG, "k=%d out of range", k);
  if (!SH || !Y || !G_old || !G_new) return tt_fail(TT_ERR_ARG, "null argument");
  {
    TTProfScope ps(p, TT_PROF_GRAM);
    TT_HIP_TRY(launch_gram(p, k, SH, Y));
  }
  TTProfScope ps(p, TT_PROF_SOLVE);
  TT_HIP_TRY(launch_prox_from_gram(p, k, static_cast<const double*>(G_old), static_cast<double*>(G_new)));
  return TT_OK;
}

tt_status tt_left_orth_absorb(tt_plan p, void* const* cores, int32_t k) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (k < 0 || k >= p->d - 1) return tt_fail(TT_ERR_ARG, "k=%d out of range [0, d-2]", k);
  if ((st = check_cores(p, cores))) return st;
  return left_orth(p, reinterpret_cast<double* const*>(cores), k);
}

tt_status tt_right_orthogonalize(tt_plan p, void* const* cores) {
  tt_status st = check_plan(p);
  if (st) return st;
  if ((st = check_cores(p, cores))) return st;
  double* const* G = reinterpret_cast<double* const*>(cores);
  for (int k = p->d - 1; k >= 1; --k)
    if ((st = right_orth(p, G, k))) return st;
  return TT_OK;
}

static tt_status residual_impl(tt_plan p, const void* X, const void* const* cores, double* out) {
  const CoreDesc cd = make_desc(p, cores);
  {
    TTProfScope ps(p, TT_PROF_RESIDUAL);
    TT_HIP_TRY(launch_residual(p, X, cd));
  }
  double host[3];
  double* dres = p->at<double>(p->o_res) + 2 * p->res_waves;
  TT_HIP_TRY(hipMemcpyAsync(host, dres, sizeof host, hipMemcpyDeviceToHost, p->stream));
  TT_HIP_TRY(hipStreamSynchronize(p->stream));
  *out = host[0];
  if (!isfinite(host[0])) return tt_fail(TT_ERR_NONFINITE, "residual is not finite (%g / %g)", host[1], host[2]);
  return TT_OK;
}

tt_status tt_residual(tt_plan p, const void* X, const void* const* cores, double* rel_residual) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (!X || !rel_residual) return tt_fail(TT_ERR_ARG, "null argument");
  if ((st = check_cores(p, cores))) return st;
  return residual_impl(p, X, cores, rel_residual);
}

tt_status tt_core_change(tt_plan p, const void* const* prev, const void* const* cur, double* change) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (!change) return tt_fail(TT_ERR_ARG, "null argument");
  if ((st = check_cores(p, prev)) || (st = check_cores(p, cur))) return st;
  double* sums = p->at<double>(p->o_chg);
  double* dout = sums + 2 * TT_MAX_ORDER;
  TT_HIP_TRY(launch_core_change(p, make_desc(p, prev), make_desc(p, cur), sums, dout));
  double host = 0.0;
  TT_HIP_TRY(hipMemcpyAsync(&host, dout, sizeof host, hipMemcpyDeviceToHost, p->stream));
  TT_HIP_TRY(hipStreamSynchronize(p->stream));
  *change = host;
  if (!isfinite(host)) return tt_fail(TT_ERR_NONFINITE, "core change is not finite (a zero or non-finite core)");
  return TT_OK;
}

// Phi_k: X contracted over modes 0..k-1 with the cores (ping-pong buffers);
// *is_x when k = 0 (Phi_0 = X).
static tt_status exact_phi(tt_plan p, const void* X, const double* const* G, int k, const void** phi, bool* is_x) {
  const void* cur = X;
  bool cur_x = true;
  char* bufs[2] = {p->ws + p->o_exphi, p->ws + p->o_exphi + p->wsize() * p->ex_phi};
  for (int i = 0; i < k; ++i) {
    TT_HIP_TRY(launch_exact_left(p, cur, cur_x, i, G[i], bufs[i & 1]));
    cur = bufs[i & 1];
    cur_x = false;
  }
  *phi = cur;
  *is_x = cur_x;
  return TT_OK;
}

static tt_status check_exact(tt_plan p, const void* X, const void* const* cores, int32_t k) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (!p->o_exphi) return tt_fail(TT_ERR_STATE, "the plan was created without TT_FLAG_EXACT");
  if (!X) return tt_fail(TT_ERR_ARG, "null X");
  if (k < 0 || k >= p->d) return tt_fail(TT_ERR_ARG, "k=%d out of range", k);
  return check_cores(p, cores);
}

tt_status tt_exact_rhs(tt_plan p, const void* X, const void* const* cores, int32_t k, void* B) {
  tt_status st = check_exact(p, X, cores, k);
  if (st) return st;
  if (!B) return tt_fail(TT_ERR_ARG, "null B");
  const double* const* G = reinterpret_cast<const double* const*>(cores);
  const void* phi;
  bool is_x;
  if ((st = exact_phi(p, X, G, k, &phi, &is_x))) return st;
  const void* Bc = nullptr;
  TT_HIP_TRY(launch_exact_right(p, phi, is_x, k, G, &Bc));
  TT_HIP_TRY(launch_exact_rhs_out(p, k, Bc, B));
  return TT_OK;
}

tt_status tt_prox_exact(tt_plan p, const void* X, void* const* cores, int32_t k, void* G_new) {
  tt_status st = check_exact(p, X, cores, k);
  if (st) return st;
  if (!G_new) return tt_fail(TT_ERR_ARG, "null G_new");
  const double* const* G = reinterpret_cast<const double* const*>(cores);
  const CoreDesc cd = make_desc(p, cores);
  const void* phi;
  bool is_x;
  const void* Bc = nullptr;
  {
    TTProfScope ps(p, TT_PROF_EXACT);
    if ((st = exact_phi(p, X, G, k, &phi, &is_x))) return st;
    TT_HIP_TRY(launch_exact_right(p, phi, is_x, k, G, &Bc));
    TT_HIP_TRY(launch_exact_grams(p, cd, k));
    TT_HIP_TRY(launch_exact_assemble(p, k, Bc, true));
  }
  TTProfScope ps(p, TT_PROF_SOLVE);
  TT_HIP_TRY(launch_prox_from_gsum(p, k, G[k], static_cast<double*>(G_new)));
  return TT_OK;
}

tt_status tt_als_sweep_exact(tt_plan p, const void* X, void* const* cores, double* rel_residual) {
  tt_status st = check_exact(p, X, cores, 0);
  if (st) return st;
  double* const* G = reinterpret_cast<double* const*>(cores);
  const int d = p->d;
  for (int k = d - 1; k >= 1; --k)
    if ((st = right_orth(p, G, k))) return st;
  const void* phi = X;
  bool is_x = true;
  char* bufs[2] = {p->ws + p->o_exphi, p->ws + p->o_exphi + p->wsize() * p->ex_phi};
  for (int k = 0; k < d; ++k) {
    {
      const void* Bc = nullptr;
      {
        TTProfScope ps(p, TT_PROF_EXACT);
        TT_HIP_TRY(launch_exact_right(p, phi, is_x, k, G, &Bc));
        // cores left of k left-orthonormal, right of k right-orthonormal: H_k^T H_k = I
        TT_HIP_TRY(launch_exact_assemble(p, k, Bc, false));
      }
      TTProfScope ps(p, TT_PROF_SOLVE);
      TT_HIP_TRY(launch_prox_from_gsum(p, k, G[k], G[k]));
    }
    if (k < d - 1) {
      if ((st = left_orth(p, G, k))) return st;
      TTProfScope ps(p, TT_PROF_EXACT);
      TT_HIP_TRY(launch_exact_left(p, phi, is_x, k, G[k], bufs[k & 1]));
      phi = bufs[k & 1];
      is_x = false;
    }
  }
  if ((st = tt_sweep_end(p))) return st;
  if (rel_residual) {
    // a failed solve (the status word) explains a non-finite residual, so it
    // is reported first
    st = residual_impl(p, X, cores, rel_residual);
    const tt_status ss = tt_plan_sync_status(p);
    return ss ? ss : st;
  }
  return TT_OK;
}

tt_status tt_plan_sync_status(tt_plan p) {
  tt_status st = check_plan(p);
  if (st) return st;
  int32_t flags[1] = {0};
  TT_HIP_TRY(hipMemcpyAsync(flags, p->ws + p->o_status, sizeof flags, hipMemcpyDeviceToHost, p->stream));
  TT_HIP_TRY(hipStreamSynchronize(p->stream));
  TT_HIP_TRY(hipMemsetAsync(p->ws + p->o_status, 0, 64, p->stream));
  if (flags[0] & 1) return tt_fail(TT_ERR_NOT_SPD, "Cholesky of SH^T SH + lambda I failed (not positive definite)");
  if (flags[0] & 2)
    return tt_fail(TT_ERR_HIP, "fused data sketch: a wave waited too long for its LDS hand-off (results invalid)");
  if (flags[0] & 4) return tt_fail(TT_ERR_ARG, "sparse sketch: a coordinate was outside [0, n_s) (entry skipped)");
  return TT_OK;
}

tt_status tt_als_sweep(tt_plan p, const void* X, void* const* cores, double* rel_residual) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (!X) return tt_fail(TT_ERR_ARG, "null X");
  if ((st = check_cores(p, cores))) return st;
  double* const* G = reinterpret_cast<double* const*>(cores);
  const int d = p->d;
  const CoreDesc cd = make_desc(p, cores);
  void* Y = p->ws + p->o_Y;
  // The data sketches need only X and this sweep's tables (generated at bind,
  // set_sweep or the end of the previous sweep, or overridden), so they run
  // ahead on the side stream while the chain of core updates proceeds on the
  // chain stream; both fork from and join back into the plan's stream.
  const bool overlap = !(p->flags & TT_FLAG_SERIAL);
  const bool fused = tt_sketch_fused01(p);
  const bool inner = tt_sketch_inner(p);
  char* Yall = p->ws + p->o_Yall;
  StreamRestore restore{p};
  // the bucket and fibre lists of every data sketch of the sweep are built
  // in one launch set ahead of the sketches, which then skip their own sorts
  struct ListsReady {
    tt_plan p;
    ~ListsReady() { p->lists_ready = false; }
  } lists_guard{p};
  auto sort_lists = [&]() -> tt_status {
    TTProfScope ps(p, TT_PROF_SKETCH_AUX);
    const hipError_t e = launch_sweep_sorts(p);
    if (e != hipSuccess) return tt_fail(TT_ERR_HIP, "key sort launch failed: %s", hipGetErrorString(e));
    p->lists_ready = true;
    return TT_OK;
  };
  if (overlap) {
    if ((st = make_streams(p))) return st;
    TT_HIP_TRY(hipEventRecord(p->ev_fork, p->user_stream));
    TT_HIP_TRY(hipStreamWaitEvent(p->side, p->ev_fork, 0));
    TT_HIP_TRY(hipStreamWaitEvent(p->chain, p->ev_fork, 0));
    p->stream = p->side;
    const int ncu = device_cus();
    const int reserved = reserved_of(p, ncu);
    p->sketch_cus = (reserved > 0 && ncu > reserved) ? ncu - reserved : 0;
    if ((st = sort_lists())) return st;
    for (int k = 0; k < d; ++k) {
      void* Yk = Yall + p->wsize() * p->J * p->tab_off[k];
      const hipError_t e = fused && k == 0   ? launch_sketch_mode0_outer(p, X, Yk)
                           : fused && k == 1 ? launch_sketch_y1_outer(p, Yk)
                           : inner && k > p->inner_m  ? hipSuccess   // written with Y_m
                           : inner && k == p->inner_m ? launch_sketch_inner(p, X, Yall)
                                             : launch_sketch_tensor(p, X, k, Yk);
      if (e != hipSuccess) return tt_fail(TT_ERR_HIP, "data sketch launch failed: %s", hipGetErrorString(e));
      TT_HIP_TRY(hipEventRecord(p->ev_y[k], p->side));
    }
    TT_HIP_TRY(hipEventRecord(p->ev_join, p->side));
    p->lists_ready = false;
    p->stream = p->chain;
    p->sketch_cus = 0;
  } else if ((st = sort_lists())) {
    return st;
  }
  if ((st = tt_sweep_begin(p, G, cd))) return st;
  for (int k = 0; k < d; ++k) {
    if ((st = tt_sweep_interface(p, cd, k))) return st;
    if (overlap) {
      Y = Yall + p->wsize() * p->J * p->tab_off[k];
      TT_HIP_TRY(hipStreamWaitEvent(p->stream, p->ev_y[k], 0));
    } else if (fused && k <= 1) {
      // Y_0 and Y_1 from the one pass, into their slots of the all-mode buffer
      Y = Yall + p->wsize() * p->J * p->tab_off[k];
      if (k == 0) {
        TT_HIP_TRY(launch_sketch_mode0_outer(p, X, Y));
        TT_HIP_TRY(launch_sketch_y1_outer(p, Yall + p->wsize() * p->J * p->tab_off[1]));
      }
    } else if (inner && k >= p->inner_m) {
      // Y_m .. Y_{d-1} from the one pass, into their slots of the all-mode buffer
      Y = Yall + p->wsize() * p->J * p->tab_off[k];
      if (k == p->inner_m) TT_HIP_TRY(launch_sketch_inner(p, X, Yall));
    } else {
      TT_HIP_TRY(launch_sketch_tensor(p, X, k, Y));
    }
    if ((st = tt_sweep_update(p, G, cd, k, Y))) return st;
  }
  p->lists_ready = false;
  if (overlap) {
    TT_HIP_TRY(hipStreamWaitEvent(p->chain, p->ev_join, 0));
    TT_HIP_TRY(hipEventRecord(p->ev_done, p->chain));
    TT_HIP_TRY(hipStreamWaitEvent(p->user_stream, p->ev_done, 0));
    p->stream = p->user_stream;
  }
  if ((st = tt_sweep_end(p))) return st;
  if (rel_residual) {
    // a failed solve (the status word) explains a non-finite residual, so it
    // is reported first
    st = residual_impl(p, X, cores, rel_residual);
    const tt_status ss = tt_plan_sync_status(p);
    return ss ? ss : st;
  }
  return TT_OK;
}

// ---------------------------------------------------------------- sketch-size policy

tt_status tt_jpolicy_features(tt_plan p, int64_t t, double last_drop, float* feats) {
  if (!p || !feats) return tt_fail(TT_ERR_ARG, "null argument");
  if (t < 0) return tt_fail(TT_ERR_ARG, "sweep index must be >= 0");
  double drop = last_drop == last_drop ? last_drop : 0.0;
  drop = drop < -1.0 ? -1.0 : (drop > 4.0 ? 4.0 : drop);
  const int d = p->d;
  for (int k = 0; k < d; ++k) {
    float* f = feats + (size_t)k * TT_JPOLICY_FEATURES;
    f[0] = (float)(log((double)p->n[k]) / 4.0);
    f[1] = (float)(log((double)p->r[k]) / 2.0);
    f[2] = (float)(log((double)p->r[k + 1]) / 2.0);
    f[3] = (float)(log((double)p->N / (double)p->n[k]) / 16.0);
    f[4] = (float)(d / 5.0);
    f[5] = (float)((double)k / d);
    f[6] = (float)((double)t / 10.0);
    f[7] = (float)drop;
  }
  return TT_OK;
}

tt_status tt_jpolicy_choose(tt_plan p, const float* params, int64_t t, double last_drop, int64_t J_min, int64_t* J,
                            double* lambda) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (!params || !J || !lambda) return tt_fail(TT_ERR_ARG, "null argument");
  if (J_min < 1 || J_min > p->J_cap) return tt_fail(TT_ERR_ARG, "J_min=%lld outside [1, %lld]", (long long)J_min,
                                                    (long long)p->J_cap);
  const int d = p->d;
  float host[TT_MAX_ORDER * (TT_JPOLICY_FEATURES + TT_JPOLICY_OUTPUTS)];
  if ((st = tt_jpolicy_features(p, t, last_drop, host))) return st;
  float* dfeat = p->at<float>(p->o_pol);
  float* dout = dfeat + TT_MAX_ORDER * TT_JPOLICY_FEATURES;
  TT_HIP_TRY(hipMemcpyAsync(dfeat, host, sizeof(float) * d * TT_JPOLICY_FEATURES, hipMemcpyHostToDevice, p->stream));
  TT_HIP_TRY(launch_mlp_forward(params, dfeat, d, dout, p->stream));
  float out[TT_MAX_ORDER * TT_JPOLICY_OUTPUTS];
  TT_HIP_TRY(hipMemcpyAsync(out, dout, sizeof(float) * d * TT_JPOLICY_OUTPUTS, hipMemcpyDeviceToHost, p->stream));
  TT_HIP_TRY(hipStreamSynchronize(p->stream));
  int best = 0;
  for (int k = 1; k < d; ++k)
    if (out[k * TT_JPOLICY_OUTPUTS] > out[best * TT_JPOLICY_OUTPUTS]) best = k;
  const double lnJ = (double)out[best * TT_JPOLICY_OUTPUTS] + 7.0;
  const double l10 = (double)out[best * TT_JPOLICY_OUTPUTS + 1] - 3.0;
  if (!isfinite(lnJ) || !isfinite(l10)) return tt_fail(TT_ERR_NONFINITE, "policy output is not finite");
  const int64_t lo = tt_floor_smooth(J_min) < J_min ? tt_round_smooth((double)J_min, J_min, p->J_cap) : J_min;
  if (p->o_exphi && lnJ >= log((double)TT_JPOLICY_EXACT_J))
    *J = 0;   // the unsketched update
  else
    *J = tt_round_smooth(exp(lnJ > 30.0 ? 30.0 : lnJ), lo, tt_floor_smooth(p->J_cap));
  // lambda stays within the range of the training labels
  const double lam = pow(10.0, l10 < TT_JPOLICY_LOG10_LAMBDA_MIN ? TT_JPOLICY_LOG10_LAMBDA_MIN
                                   : (l10 > TT_JPOLICY_LOG10_LAMBDA_MAX ? TT_JPOLICY_LOG10_LAMBDA_MAX : l10));
  *lambda = lam;
  return TT_OK;
}

tt_status tt_plan_fallback_J(tt_plan p, double eps, double delta, int64_t* J) {
  if (!p || !J) return tt_fail(TT_ERR_ARG, "null argument");
  double m = 0.0;
  for (int k = 0; k < p->d; ++k) {
    double mk = 0.0;
    tt_status st = tt_sketch_size_bound(p->r[k] * p->r[k + 1], p->d - 1, eps, delta, &mk);
    if (st) return st;
    if (mk > m) m = mk;
  }
  const double cap = (double)p->J_cap;
  *J = tt_floor_smooth(m < cap ? (int64_t)ceil(m) : p->J_cap);
  return TT_OK;
}

tt_status tt_als_run(tt_plan p, const void* X, void* const* cores, const float* params, int32_t max_sweeps, double target,
                     int64_t J_min, double* residuals, int64_t* Js, double* lambdas, tt_run_stats* stats) {
  tt_status st = check_plan(p);
  if (st) return st;
  if (!X || !stats) return tt_fail(TT_ERR_ARG, "null argument");
  if (max_sweeps < 1) return tt_fail(TT_ERR_ARG, "max_sweeps must be >= 1");
  if ((st = check_cores(p, cores))) return st;
  stats->sweeps = 0;
  stats->reached = 0;
  stats->fallbacks = 0;
  stats->residual = 1.0;
  double prev = 1.0, drop = 0.0;
  bool fallback = false;
  // the exact sweep replaces the sketched fallback when the plan can run it
  // and the Corollary 3 size of some core update is no smaller than that
  // update's unsketched problem (N / n_k rows)
  bool exact_fb = false;
  if (p->o_exphi) {
    for (int k = 0; k < p->d; ++k) {
      double m = 0.0;
      if ((st = tt_sketch_size_bound(p->r[k] * p->r[k + 1], p->d - 1, 0.5, 0.1, &m))) return st;
      if (m >= (double)(p->N / p->n[k])) exact_fb = true;
    }
  }
  for (int32_t t = 0; t < max_sweeps; ++t) {
    bool exact = false;
    if (params) {
      int64_t J = p->J;
      double lam = p->lambda;
      if (fallback) {
        if ((st = tt_plan_fallback_J(p, 0.5, 0.1, &J))) return st;
        lam = p->lambda0;
        stats->fallbacks += 1;
        exact = exact_fb;
      } else if ((st = tt_jpolicy_choose(p, params, t, t == 0 ? 0.0 : drop, J_min, &J, &lam))) {
        return st;
      } else if (J == 0) {
        exact = true;     // the policy chose the unsketched update
        J = p->J;
      }
      if (J != p->J || lam != p->lambda)
        if ((st = tt_plan_set_sketch(p, J, lam))) return st;
    }
    if (Js) Js[t] = exact ? 0 : p->J;
    if (lambdas) lambdas[t] = p->lambda;
    double res = 0.0;
    if ((st = exact ? tt_als_sweep_exact(p, X, cores, &res) : tt_als_sweep(p, X, cores, &res))) return st;
    if (residuals) residuals[t] = res;
    stats->sweeps = t + 1;
    stats->residual = res;
    drop = log10(prev / res);
    // the residual check: a sweep that does not lower the previous sweep's
    // residual sends the next one to the fallback size.  The first sweep has
    // no measured predecessor (the 1.0 above only seeds the drop feature; a
    // random start can lie above 1), so the check begins with the second.
    fallback = params && t > 0 && !(res < prev);
    prev = res;
    if (res <= target) {
      stats->reached = 1;
      break;
    }
  }
  return TT_OK;
}

}  // extern "C"
