// Internal declarations of the TT-TensorSketch HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/tt_sketch.h"

// Packed hash key: bits 0..30 bucket in [0, J), bit 31 sign (1 = negative).
#define TT_KEY_MASK 0x7fffffffu
#define TT_KEY_SIGN 0x80000000u

struct tt_plan_s {
  int d;
  int64_t n[TT_MAX_ORDER];
  int64_t r[TT_MAX_ORDER + 1];
  int64_t J;
  double lambda;
  uint64_t seed;
  tt_dtype xdt, wdt;
  int gram_mode;
  hipStream_t stream;          // stream the launchers enqueue on (the user's, or the side stream)
  hipStream_t user_stream;     // the plan's stream (tt_sketch_plan / tt_plan_set_stream)
  hipStream_t side;            // plan-owned stream for the overlapped data sketches (lazy)
  hipStream_t chain;           // plan-owned stream for the rest of an overlapped sweep (lazy)
  hipEvent_t ev_fork, ev_join, ev_done, ev_y[TT_MAX_ORDER];
  int64_t J_cap;               // J of the plan descriptor: workspace sized for it
  const int64_t* dsweep;       // device sweep counter read by the table generator (batched graphs), or null
  double lambda0;              // lambda of the plan descriptor
  int32_t reserved_cus;        // CUs withheld from the side stream (its CU mask)
  int32_t sketch_cus;          // CUs a persistent sketch grid may fill on p->stream (0: all)
  uint32_t flags;
  int64_t sweep;
  bool override_tables;

  // derived sizes
  int64_t N;                   // entries of X
  int64_t tab_off[TT_MAX_ORDER + 1];   // prefix of n (packed table offsets)
  int64_t max_n, s_max, r_max;
  int64_t max_M, max_R;        // largest inner / outer fibre-key table
  int64_t O0;                  // outer combos for k = 0 (modes 2..d-1)
  int inner_m;                 // inner sketch over modes 0..inner_m-1 (Y_k, k >= inner_m, from it); 0: none
  int64_t inner_rows;          // rows of one of its slabs: n_1 ... n_{inner_m - 1}
  int64_t inner_O;             // its slabs: n_{inner_m} ... n_{d-1}
  int64_t part_entries;        // data-sketch partial accumulators (work type elements)
  int64_t gram_chunks;         // split-K chunks of the Gram
  int64_t chat_cols;           // sum_i R_i R_{i+1}
  int64_t qr_m;                // max rows of a QR operand
  int fft_radix[32];
  int fft_nrad;
  int64_t res_waves;

  // workspace
  char* ws;
  size_t ws_bytes;
  size_t ws_need;
  void* prof;                  // ProfState* when measurement is enabled, else null

  size_t o_tab, o_KI, o_KO, o_cnt, o_hist, o_sortO, o_part, o_chat, o_pre, o_suf, o_SH, o_Y,
      o_gram, o_minv, o_W, o_qrA, o_qrQ, o_qrR, o_status, o_res, o_gold, o_Yall, o_pol, o_gsum, o_resU, o_resH,
      o_tw, o_zo,                  // o_zo: outer sketch of the fused k = 0 pass (0: not fused)
      o_zi,                        // o_zi: inner sketch Z of the k >= 2 pass (0: not used)
      o_zperm;                     // buckets of the joint k = 0 pass, largest first (J_cap entries)
  // exact update (TT_FLAG_EXACT; 0 otherwise): two left-interface buffers of
  // ex_phi work-type values, two right-chain buffers of ex_chain, ex_part FP64
  // slice partials, the two Gram factors (2 x 256 doubles)
  size_t o_exphi, o_exch, o_expart, o_exgram;
  size_t o_exmerge;            // the last two cores merged (FP64), 0: not used
  size_t o_spacc;              // FP64 accumulators of the sparse sketches (J_cap x sum n)
  size_t o_chg;                // core change: 2 d partial sums and the result (FP64)
  int64_t ex_phi, ex_chain, ex_part;
  int64_t tw_J;                // J whose roots of unity the o_tw table holds (0: none)
  // key sorts, slot 0 = outer tuples of the k = 0 sketch, slot k >= 1 =
  // fibres of mode k: keys (o_skeys), per-chunk counts (o_hist), fibre lists
  // (o_flist, uint2) and their offsets (o_foff, J_cap + 1 per slot)
  size_t o_skeys, o_flist, o_foff;
  int64_t skeys_off[TT_MAX_ORDER], flist_off[TT_MAX_ORDER], hist_off[TT_MAX_ORDER];
  bool lists_ready;            // this sweep's lists are built (the sketches skip their sorts)

  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  size_t wsize() const { return wdt == TT_F64 ? 8 : 4; }
  size_t xsize() const { return xdt == TT_F64 ? 8 : (xdt == TT_F32 ? 4 : 2); }
};

// Error plumbing ------------------------------------------------------------
void tt_set_error(const char* fmt, ...);
tt_status tt_fail(tt_status st, const char* fmt, ...);
#define TT_HIP_TRY(expr)                                                         \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return tt_fail(TT_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Measurement scopes (no-ops unless tt_plan_profile enabled them)
void tt_prof_begin(const tt_plan_s* p, int cls);
void tt_prof_end(const tt_plan_s* p, int cls);
void tt_prof_free(tt_plan_s* p);
struct TTProfScope {
  const tt_plan_s* p;
  int cls;
  TTProfScope(const tt_plan_s* p_, int c) : p(p_), cls(c) { tt_prof_begin(p, cls); }
  ~TTProfScope() { tt_prof_end(p, cls); }
};

// Per-core launch descriptor (passed by value to kernels).
struct CoreDesc {
  const double* G[TT_MAX_ORDER];
  int32_t r0[TT_MAX_ORDER], n[TT_MAX_ORDER], r1[TT_MAX_ORDER];
  int32_t tab_off[TT_MAX_ORDER];
  int64_t chat_off[TT_MAX_ORDER];   // column offset of core i in the transformed-core store
  int32_t d;
};

// One problem's interface step in the batched form (FP32): core descriptor
// and plan buffers; k = the step (the transform of core k - 1 precedes it
// for k >= 1, over cols columns), s = R_k R_{k+1} output columns.
struct BIface {
  CoreDesc cd;
  const uint32_t* tab;
  void* chat;
  void* pre;
  void* suf;
  void* SH;
  const void* tw;
  uint64_t fft_code;   // the problem's FFT radices, 4 bits each
  int32_t fft_nrad, J;
  int32_t k, cols, s;
};
// Jmax: the largest J of the batch (LDS and chain grid)
hipError_t launch_interface_batched(const void* desc, int32_t nprob, int32_t k, int32_t Jmax, int32_t max_cols,
                                    int32_t max_s, int32_t cw, hipStream_t st);

// Launchers (each enqueues on p->stream; returns hipSuccess or the launch error)
hipError_t launch_gen_tables(const tt_plan_s* p, int64_t sweep);
// batched table generation (the sweep index from each plan's device counter)
size_t tt_tab_args_bytes();
hipError_t tt_tab_args(const tt_plan_s* p, void* out);
hipError_t launch_gen_tables_batched(const void* args, int32_t nprob, int64_t max_entries, hipStream_t st);
hipError_t launch_fill_twiddles(const tt_plan_s* p);   // o_tw <- exp(-2 pi i e / J), e < J
hipError_t launch_build_keys(const tt_plan_s* p, uint32_t* out, int64_t count, int first, int last);
hipError_t launch_build_keys_modes(const tt_plan_s* p, uint32_t* out, int64_t count, const int* modes, int nm);
hipError_t launch_outer_sort(const tt_plan_s* p);     // k = 0 bucket lists (modes 2..d-1)
hipError_t launch_fibre_sort(const tt_plan_s* p, int k);   // k >= 1 fibre lists by key
int64_t tt_sort_chunks(int64_t count);                     // workgroups of a key sort of count tuples
hipError_t launch_sweep_sorts(const tt_plan_s* p);         // every list of one sweep's data sketches
const uint2* tt_fibre_list(const tt_plan_s* p, int k);     // the k >= 1 fibre list of mode k
size_t tt_sort_args_bytes();                               // one argument set of the key sorts
hipError_t tt_sort_args_outer(const tt_plan_s* p, void* out, int32_t* nb);   // plan p's outer sort, host memory
hipError_t tt_sort_args_slabs(const tt_plan_s* p, int k, void* out, int32_t* nb);   // mode-k slab sort (k >= 2)
hipError_t launch_outer_sorts_batched(const void* args, const void* src, int32_t nsets, int32_t nblocks, int32_t J,
                                      hipStream_t st);
hipError_t launch_sketch_tensor(const tt_plan_s* p, const void* X, int k, void* Y);
// sparse sketch (k_sparse.hip): k >= 0 one mode, k < 0 every mode
hipError_t launch_sketch_sparse(const tt_plan_s* p, int64_t nnz, const int32_t* coords, const void* vals, int k,
                                void* Y);
// exact update (k_exact.hip)
void tt_exact_sizes(const tt_plan_s* p, int64_t* phi, int64_t* chain);
int64_t tt_exact_merge_doubles(const tt_plan_s* p);
hipError_t launch_exact_left(const tt_plan_s* p, const void* phi_k, bool is_x, int k, const double* Gk, void* phi_next);
hipError_t launch_exact_right(const tt_plan_s* p, const void* phi_k, bool is_x, int k, const double* const* G,
                              const void** result);
hipError_t launch_exact_grams(const tt_plan_s* p, const CoreDesc& cd, int k);
hipError_t launch_exact_assemble(const tt_plan_s* p, int k, const void* Bc, bool use_grams);
hipError_t launch_exact_rhs_out(const tt_plan_s* p, int k, const void* Bc, void* B);
// Y_0 and Y_1 from one pass over X: the fused k = 0 pass (Y_0 and the outer
// sketch in o_zo), then Y_1 from the outer sketch
hipError_t launch_sketch_mode0_outer(const tt_plan_s* p, const void* X, void* Y0);
hipError_t launch_sketch_y1_outer(const tt_plan_s* p, void* Y1);
bool tt_sketch_fused01(const tt_plan_s* p);
// Y_k for all k >= 2 from one pass over X through the inner sketch Z (o_zi),
// into their slots of the all-mode buffer Yall
hipError_t launch_sketch_inner(const tt_plan_s* p, const void* X, void* Yall);
bool tt_sketch_inner(const tt_plan_s* p);
int64_t tt_inner_slices(const tt_plan_s* p, int k);   // workgroups per column of the Y_k-from-Z stage
// the k = 0 pass writes the inner sketch too (FP32 work): vectors per thread
// of its kernel (0: not taken), whether the plan takes it, and whether it runs
// for this X (16-byte aligned)
int tt_joint_vectors(const tt_plan_s* p);
bool tt_sketch_joint(const tt_plan_s* p);
bool tt_sketch_joint_ok(const tt_plan_s* p, const void* X);
int64_t tt_outer_slices(const tt_plan_s* p);   // workgroups per column of the Y_1 stage
hipError_t launch_core_fft(const tt_plan_s* p, const CoreDesc& cd, int core_lo, int core_hi, int skip);
hipError_t launch_interface_from_chat(const tt_plan_s* p, const CoreDesc& cd, int k, void* SH);
hipError_t launch_gram(const tt_plan_s* p, int k, const void* SH, const void* Y);
hipError_t launch_prox_from_gram(const tt_plan_s* p, int k, const double* G_old, double* G_new);
// the solve alone, from [M | B] already in o_gsum (row-major s x (s + n_k))
hipError_t launch_prox_from_gsum(const tt_plan_s* p, int k, const double* G_old, double* G_new);
hipError_t launch_qr_core(const tt_plan_s* p, double* G, int64_t m, int64_t rcols, int64_t rs, int64_t cs);
hipError_t launch_absorb_left(const tt_plan_s* p, double* Gnext, int64_t r, int64_t cols);   // G^R <- R G^R
hipError_t launch_absorb_right(const tt_plan_s* p, double* Gprev, int64_t rows, int64_t r);  // G^L <- G^L R^T
hipError_t launch_residual(const tt_plan_s* p, const void* X, const CoreDesc& cd);
hipError_t launch_core_change(const tt_plan_s* p, const CoreDesc& prev, const CoreDesc& cur, double* sums,
                              double* out);
int64_t tt_residual_waves(int64_t O0, int64_t n1);   // waves (and partials) of the residual pass
hipError_t launch_copy_f64(const tt_plan_s* p, double* dst, const double* src, int64_t count);

#define TT_SKETCH_MAX_WG 4096
// CUs an overlapped sweep keeps free of the data sketches by default
#ifndef TT_DEFAULT_RESERVED_CUS
#define TT_DEFAULT_RESERVED_CUS (-1)   // -1: the CUs of one XCD (CU count / 8), else 0
#endif
int64_t tt_sketch_workgroups(const tt_plan_s* p, int k, int64_t resident);   // k >= 1 sketch grid
int64_t tt_sketch_slots(const tt_plan_s* p, int k, int64_t W);              // partials per column
bool tt_sketch_use_gs(const tt_plan_s* p, int k);                           // key-grouped k >= 1 path
int64_t tt_gram_chunks(int64_t J);                      // split-K chunks of the Gram

// Allow a kernel more than 64 KB of dynamic LDS (gfx950 has 160 KB per CU).
template <typename K>
inline hipError_t tt_allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// FFT plan helper: factor J into radices {4,2,3,5,7}; returns false if J has other factors.
bool tt_factor_fft(int64_t J, int* radix, int* nrad);

// One problem's core update k within a batched step (FP32 work): the device
// array of these drives the batched Gram, solve, QR and absorb launches
// (batch.hip), one workgroup (or block set) per problem.
// Global-address-space pointers: kernels that take their buffers from a
// descriptor in memory see generic pointers, which compile to flat accesses
// sharing the LDS wait counter; casting to these keeps them global.
typedef double __attribute__((address_space(1)))* gdbl;
typedef const double __attribute__((address_space(1)))* cgdbl;
typedef int32_t __attribute__((address_space(1)))* gi32;

struct BUpd {
  const float* SH;      // J x s
  const float* Y;       // J x n_k
  double* gpart;        // Gram partials (FP64 MFMA accumulators)
  double* gsum;         // summed Gram
  double* Lg;           // Cholesky factor
  int32_t* status;      // plan status words
  double* G;            // core k (updated in place)
  double* Gnext;        // core k + 1 (R absorbed), or null for k = d - 1
  double* R;            // QR factor R
  double lambda;
  int32_t J, s, nk, rk, rk1, chunks, CB, ncols_next;   // ncols_next = n_{k+1} R_{k+2}
  int32_t kchunk;       // Gram K-chunk (rows of SH per partial); chunks = ceil(J / kchunk)
};
hipError_t launch_gram_batched(const BUpd* d, int32_t nprob, int32_t gx, hipStream_t st);
hipError_t launch_gram_sum_batched(const BUpd* d, int32_t nprob, int32_t max_count, hipStream_t st);
int32_t tt_gram_chunk_min();   // the K-chunk the single-plan Gram uses (partial buffers are sized for it)
size_t tt_chol_lds_bytes(int64_t s);   // dynamic LDS of the Cholesky kernel for an s x s system
int64_t tt_chol_out_doubles(int64_t s);  // packed L plus the inverses of its 16 x 16 diagonal blocks
hipError_t launch_solve_batched(const BUpd* d, int32_t nprob, int32_t max_s, int32_t max_count, int32_t max_cb_blocks,
                                size_t lds_chol, size_t lds_trsm, hipStream_t st);
hipError_t launch_qr_batched(const BUpd* d, const int32_t* idx, int32_t nidx, int32_t rmax, int32_t rpt, hipStream_t st);
hipError_t launch_absorb_left_batched(const BUpd* d, int32_t nprob, int32_t max_cols, hipStream_t st);

// One problem's step of the right-to-left orthogonalisation in the batched
// form: QR of G_s^R transposed (m = n_s R_{s+1} rows, r = R_s columns, G_s
// itself with row stride r), then G_{s-1} (rows = R_{s-1} n_{s-1} x r) <-
// G_{s-1} R^T.  Gprev is null for a problem whose QR runs on its own.
struct BRo {
  double* G;
  double* Gprev;
  double* R;
  int32_t m, r, rows;
};
hipError_t launch_qr_right_batched(const BRo* d, const int32_t* idx, int32_t nidx, int32_t rmax, int32_t rpt,
                                   hipStream_t st);
hipError_t launch_absorb_right_batched(const BRo* d, int32_t nprob, int32_t max_rows, hipStream_t st);
// the transforms of cores 1..d-1 of every problem (the descriptors of step 0)
hipError_t launch_core_fft_batched(const void* desc, int32_t nprob, int32_t Jmax, int32_t max_cols, hipStream_t st);

// pieces of one sweep (api.hip), shared by tt_als_sweep and the batched driver
CoreDesc tt_make_desc(const tt_plan_s* p, const void* const* cores);
tt_status tt_sweep_begin(tt_plan p, double* const* G, const CoreDesc& cd);
tt_status tt_sweep_interface(tt_plan p, const CoreDesc& cd, int k);
tt_status tt_sweep_update(tt_plan p, double* const* G, const CoreDesc& cd, int k, const void* Y);
tt_status tt_sweep_end(tt_plan p);
tt_status tt_plan_check(tt_plan p);

// sketch-size policy (k_mlp.hip)
hipError_t launch_mlp_forward(const float* params, const float* feats, int32_t B, float* out, hipStream_t stream);
int64_t tt_round_smooth(double x, int64_t lo, int64_t hi);   // nearest 2^a 3^b 5^c 7^e in [lo, hi]
int64_t tt_floor_smooth(int64_t x);                          // largest 2^a 3^b 5^c 7^e <= x
