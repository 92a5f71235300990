/*
 * tt_sketch.h -- C ABI of the MI355X (gfx950) implementation of randomized
 * proximal TT-ALS with TensorSketch (TT-TS): Chen, Jiang, Yu, Qi,
 * "Low-rank Tensor Train Decomposition Using TensorSketch", arXiv 2309.08093.
 *
 * Problem statement (Algorithm 1, Sec. 3): given a tensor A (here X) with mode
 * sizes n_0..n_{d-1}, TT ranks R_0..R_d (R_0 = R_d = 1), sketch size J (the
 * paper's m) and proximal parameter lambda (the paper's sigma), compute TT
 * cores G_k of shape (R_k, n_k, R_{k+1}) by sweeps of sketched proximal
 * least-squares updates.
 *
 * Conventions shared by every entry point
 *   - Indices are 0-based.  X is dense, mode 0 varying fastest (the paper's
 *     linear order, Sec. 2.2), i.e. a row-major torch tensor of shape
 *     (n_{d-1}, ..., n_0).
 *   - Core k is FP64, shape (R_k, n_k, R_{k+1}), first index fastest:
 *     G_k(a, i, b) at a + R_k * (i + n_k * b).  Its left unfolding G^L
 *     (R_k n_k x R_{k+1}) and right unfolding G^R (R_k x n_k R_{k+1}) (Sec. 1.2)
 *     are column-major views of the same memory.
 *   - "Work" arrays (Y, SH) use the plan's work type (FP64 or FP32) and are
 *     column-major: Y_k is J x n_k at Y[b + J*i], SH_k is J x R_k R_{k+1} at
 *     SH[b + J*(a + R_k*c)] (column alpha + beta R_k, Theorem 1, Sec. 3).
 *   - Ownership: the caller owns every device buffer it passes (X, cores, Y,
 *     SH, workspace) and the stream.  The library never allocates or frees
 *     device memory; all device scratch lives in the caller's workspace.
 *   - Asynchrony: every call enqueues work on the plan's stream and returns.
 *     Only tt_plan_get_tables, tt_plan_sync_status and a non-NULL
 *     rel_residual synchronise the stream.
 *   - Errors: argument and shape errors return before any device work, with
 *     outputs untouched.  A failed launch returns TT_ERR_HIP.  A failed
 *     Cholesky (not SPD, e.g. lambda = 0 with a rank-deficient SH) is recorded
 *     on the device and reported by the next synchronising call as
 *     TT_ERR_NOT_SPD.  Nothing throws across the ABI and nothing prints;
 *     tt_last_error() returns a thread-local message for the last failure.
 *   - A plan is not thread-safe; use one plan per stream.
 */
#ifndef TT_SKETCH_H
#define TT_SKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_MAX_ORDER 16      /* d */
#define TT_MAX_J 8192        /* sketch size (LDS FFT and bucket accumulators) */
#define TT_MAX_RANK 16       /* max R_k */
#define TT_MAX_S 180         /* max R_k R_{k+1} (packed FP64 Cholesky in LDS) */
#define TT_MAX_N0 4096       /* max n_0 */

typedef struct tt_plan_s* tt_plan;

typedef enum {
  TT_OK = 0,
  TT_ERR_ARG = 1,        /* null pointer, bad enum, k out of range, bad J / lambda */
  TT_ERR_SHAPE = 2,      /* infeasible ranks or sizes beyond the limits above */
  TT_ERR_WORKSPACE = 3,  /* no workspace bound, or smaller than required */
  TT_ERR_HIP = 4,        /* a HIP runtime call or kernel launch failed */
  TT_ERR_NOT_SPD = 5,    /* Cholesky of SH^T SH + lambda I failed */
  TT_ERR_NONFINITE = 6,  /* NaN/Inf in a residual, a core change or a solve */
  TT_ERR_STATE = 7       /* call order violated (e.g. tables never set) */
} tt_status;

typedef enum { TT_F64 = 0, TT_F32 = 1, TT_BF16 = 2 } tt_dtype;

typedef enum {
  TT_GRAM_WORK = 0,      /* Gram / RHS contractions in the work type (FP32 or FP64 MFMA) */
  TT_GRAM_BF16 = 1       /* SH and Y rounded to BF16, MFMA with FP32 accumulation */
} tt_gram_mode;

typedef struct {
  int32_t d;             /* tensor order, 2 <= d <= TT_MAX_ORDER */
  const int64_t* n;      /* d mode sizes (host memory, read during the call only) */
  const int64_t* r;      /* d+1 TT ranks, r[0] = r[d] = 1, r[k] <= r[k-1] n[k-1], r[k] <= n[k] r[k+1] */
  int64_t J;             /* sketch size m, 1 <= J <= TT_MAX_J, prime factors in {2,3,5,7} */
  double lambda;         /* proximal parameter sigma >= 0 */
  uint64_t seed;         /* seed of the hash/sign tables */
  tt_dtype x_dtype;      /* storage type of X */
  tt_dtype work_dtype;   /* TT_F64 or TT_F32: type of Y, SH and the sketch accumulators */
  int32_t gram_mode;     /* tt_gram_mode */
  uint32_t flags;        /* TT_FLAG_* bits, 0 for the defaults */
} tt_plan_desc;

/* tt_als_sweep runs the d data sketches of a sweep (which need only X and the
 * sweep's tables) on a second, plan-owned stream of default priority,
 * overlapped with the latency-bound interface / solve / QR chain on the
 * plan's stream, joined by events.  This flag keeps every kernel on the
 * plan's stream instead. */
#define TT_FLAG_SERIAL 1u

/* Data sketches of a sweep (Algorithm 1 draws S once per outer iteration, so
 * all d sketches share the tables).  When d >= 3 the k = 0 pass over X can
 * be the TensorSketch of X over modes 2..d-1 (J x n_0 x n_1 values of the
 * work type in the workspace), from which Y_0 and Y_1 follow without their
 * own passes over X.  By default this is done when that intermediate is
 * small, 2 J n_0 n_1 sizeof(work) <= N sizeof(X) / 2.  TT_FLAG_FUSE asks for
 * it whenever d >= 3, TT_FLAG_NO_FUSE never (not both).  tt_sketch_tensor(k)
 * is not affected: it always makes its own pass. */
#define TT_FLAG_FUSE 2u
#define TT_FLAG_NO_FUSE 4u

/* Data sketches of modes k >= m (d >= 4, n_0 <= 1024, 2 <= m <= d-2): the
 * pass of mode m can instead write the TensorSketch of every slab
 * X(:, ..., :, o) over modes 0..m-1 alone (Z: J x prod(n_m..n_{d-1}) values
 * of the work type in the workspace; row o holds
 * sum v_0(i_0)...v_{m-1}(i_{m-1}) X(i_0, ..., i_{m-1}, o) at bucket
 * (h_0(i_0) + ... + h_{m-1}(i_{m-1})) mod J).  Y_k for every k >= m follows
 * from Z by the TensorSketch over the remaining modes (a cyclic shift of
 * each row by their bucket, times their sign), so one pass over X serves all
 * of them; the modes 2..m-1 keep their own passes.  The plan takes the m
 * with the fewest bytes moved, (m - 2) N sizeof(X) + N max(sizeof(X), 4) +
 * (d - m + 1) |Z| sizeof(work) (the pass that writes Z adds each entry by an
 * LDS atomic, which costs about the time of 4 bytes of HBM), among those
 * whose slab rows (n_1 ... n_{m-1}) number at most 16384, and by default
 * uses it when that is at most 0.75 (d - 2) N sizeof(X).  TT_FLAG_INNER asks for it whenever d >= 4 and n_0 <= 1024,
 * TT_FLAG_NO_INNER never (not both).  Independent of TT_FLAG_FUSE;
 * tt_sketch_tensor(k) is not affected.  With both intermediates, m = 2, FP32 work,
 * FP32 or BF16 X, n_0 a multiple of 16 bytes' worth of X values and slabs
 * of at most 40960 values, the k = 0 pass writes Z as well (one pass over X
 * per sweep) whenever X is 16-byte aligned. */
#define TT_FLAG_INNER 16u
#define TT_FLAG_NO_INNER 32u

/* Workspace for the exact (unsketched) update: tt_exact_rhs, tt_prox_exact,
 * tt_als_sweep_exact, and the exact fallback sweep of tt_als_run.  Adds two
 * buffers of max_k R_k n_k ... n_{d-1} and two of the largest right-chain
 * intermediate (about R N / n_{d-1}) work-type values. */
#define TT_FLAG_EXACT 8u

/* Create a plan (Algorithm 1, REQUIRE line: tensor shape, TT ranks, m, sigma).
 * Validates the descriptor, computes the workspace size the caller must
 * provide (*workspace_bytes), and stores the stream (a hipStream_t, may be
 * NULL for the null stream).  Launches nothing.  The sweep index starts at 0
 * and the tables are generated when the workspace is bound. */
tt_status tt_sketch_plan(const tt_plan_desc* desc, void* hip_stream,
                         size_t* workspace_bytes, tt_plan* out);

/* Bind caller-owned device memory of at least *workspace_bytes bytes,
 * 256-byte aligned.  Enqueues the generation of the sweep-0 tables. */
tt_status tt_plan_bind_workspace(tt_plan plan, void* dev_workspace, size_t bytes);

tt_status tt_plan_set_stream(tt_plan plan, void* hip_stream);
tt_status tt_plan_destroy(tt_plan plan);

/* TensorSketch operators S_s for sweep t (Algorithm 1, "Define TensorSketch
 * operators", once per outer iteration; Sec. 2.2 Definitions of CountSketch
 * and TensorSketch).  For every mode s, h_s[i] in [0, J) and v_s[i] in {-1,+1}
 * are drawn from SplitMix64 keyed by seed XOR ((t+1)*2^16 + s): state0 =
 * mix64(key); output j = mix64(state0 + (j+1)*0x9E3779B97F4A7C15);
 * h_s[i] = floor(out_i * J / 2^64), v_s[i] = 1 - 2*(out_{n_s+i} >> 63).
 * Generated on the device; clears any table override. */
tt_status tt_plan_set_sweep(tt_plan plan, int64_t t);
tt_status tt_plan_get_sweep(tt_plan plan, int64_t* t);

/* Change the sketch size and proximal parameter used from now on (Alg. 1
 * takes m and sigma as inputs; a sketch-size policy may change them between
 * sweeps).  1 <= J <= the descriptor's J (the workspace is sized for it) and
 * J a product of 2, 3, 5 and 7; lambda finite and >= 0.  Regenerates the
 * tables of the current sweep for the new J and drops any table override.
 * TT_ERR_ARG otherwise, with the plan unchanged. */
tt_status tt_plan_set_sketch(tt_plan plan, int64_t J, double lambda);
tt_status tt_plan_get_sketch(tt_plan plan, int64_t* J, double* lambda);

/* Copy the current tables of mode s to host memory (n_s entries each).
 * Synchronises the stream. */
tt_status tt_plan_get_tables(tt_plan plan, int32_t s, int32_t* h, int8_t* v);

/* Override the tables of mode s with host values (h in [0, J), v = +-1).
 * The override persists until tt_plan_set_sweep; tt_als_sweep keeps it
 * (used for the paper's worked example and for injective test sketches). */
tt_status tt_plan_set_tables(tt_plan plan, int32_t s, const int32_t* h, const int8_t* v);

/* Data sketch Y_k = S_{-k} A_(k)^T (sketched subproblem, Sec. 3 (lrtt_sub4);
 * TensorSketch over all modes except k, (eqn_h)-(eqn_v)): every entry
 * X(i_0..i_{d-1}) adds prod_{s!=k} v_s(i_s) X(i) to
 * Y[(sum_{s!=k} h_s(i_s)) mod J, i_k].  X: device, x_dtype, N entries.
 * Y: device, work type, J x n_k column-major, fully overwritten. */
tt_status tt_sketch_tensor(tt_plan plan, const void* X, int32_t k, void* Y);

/* All d data sketches of the current sweep's tables, Y_k = S_{-k} A_(k)^T
 * for k = 0..d-1 ((lrtt_sub4), Algorithm 1's sketches of one outer
 * iteration), with as few passes over X as the plan allows (TT_FLAG_FUSE).
 * Yall: device, work type; Y_k is J x n_k column-major at element offset
 * J (n_0 + ... + n_{k-1}); fully overwritten.  Same errors as
 * tt_sketch_tensor. */
tt_status tt_sketch_tensor_all(tt_plan plan, const void* X, void* Yall);

/* Data sketch of a sparse tensor in O(nnz) (Sec. 3, complexity remark after
 * Theorem 3): the same Y_k = S_{-k} A_(k)^T as tt_sketch_tensor, from the
 * nonzeros only.  COO input: coords device int32, nnz x d row-major
 * (coords[e d + s] = i_s of nonzero e), vals device x_dtype (nnz values);
 * repeated coordinates add.  Y: device work type, J x n_k column-major, fully
 * overwritten (zero for nnz = 0).  tt_sketch_sparse_all reads each nonzero
 * once and writes every Y_k, at element offset J (n_0 + ... + n_{k-1}) of
 * Yall.  Sums are FP64.  A coordinate outside [0, n_s) makes its entry be
 * skipped and the next synchronising call return TT_ERR_ARG. */
tt_status tt_sketch_sparse(tt_plan plan, int64_t nnz, const int32_t* coords, const void* vals, int32_t k, void* Y);
tt_status tt_sketch_sparse_all(tt_plan plan, int64_t nnz, const int32_t* coords, const void* vals, void* Yall);

/* How tt_sketch_tensor_all and tt_als_sweep obtain each Y_k (host query, no
 * device work): src[k] = k when Y_k takes its own pass over X, src[k] = j != k
 * when it is derived from an intermediate written by the pass of mode j
 * (src[1] = 0 with the outer sketch of TT_FLAG_FUSE, src[k] = m for k > m
 * with the inner sketch of TT_FLAG_INNER, src[k] = 0 for every k >= 1 when
 * the k = 0 pass writes both; a 16-byte aligned X is assumed for the last).
 * src: host array of d entries. */
tt_status tt_plan_sketch_sources(tt_plan plan, int32_t* src);

/* Interface sketch SH_k = S_{-k} (G_{>k}^T (x) G_{<k}) (Theorem 1 and 2,
 * Sec. 3): per-core CountSketch along mode 2, length-J FFT, slice-wise
 * products per frequency, face-splitting product, inverse FFT, real part.
 * cores: host array of d device pointers to FP64 cores (core k unused).
 * SH: device, work type, J x R_k R_{k+1} column-major, fully overwritten. */
tt_status tt_sketch_interface(tt_plan plan, const void* const* cores, int32_t k, void* SH);

/* Sketched proximal update of core k (closed form, Sec. 3 (ite), with
 * S^T S): G_k(2)^new = (Y^T SH + lambda G_k(2)^old)(SH^T SH + lambda I)^{-1}.
 * SH, Y: device, work type (as produced above).  G_old, G_new: device FP64
 * cores of shape (R_k, n_k, R_{k+1}); they may alias.  The Gram and RHS
 * contractions run on MFMA (work type, or BF16 with FP32 accumulation under
 * TT_GRAM_BF16); the Cholesky factorisation and the solve run in FP64. */
tt_status tt_prox_solve(tt_plan plan, int32_t k, const void* SH, const void* Y,
                        const void* G_old, void* G_new);

/* Exact proximal update (Sec. 3, (lrtt_sub_prox), whose closed form is (ite)
 * with S = I): the plan needs TT_FLAG_EXACT (TT_ERR_STATE otherwise).
 *
 * tt_exact_rhs: B = A_(k) H_k with H_k = G_{>k}^T (x) G_{<k} (defined under
 * (lrtt_sub4)), n_k x R_k R_{k+1}, column-major, work type:
 * B[i + n_k (alpha + R_k beta)].  X is contracted with the cores one mode at
 * a time (left interface over modes 0..k-1, then modes d-1..k+1): one pass
 * over X and intermediates of at most about R N / n_i values; H_k is never
 * formed.  cores: host array of d device pointers (core k unused).
 *
 * tt_prox_exact: G_k(2)^new = (A_(k) H_k + lambda G_k(2)^old)
 * (H_k^T H_k + lambda I)^{-1} with H_k^T H_k = (G_{>k} G_{>k}^T) (x)
 * (G_{<k}^T G_{<k}) from the cores, FP64 Cholesky and substitution.  G_old =
 * cores[k]; G_new may alias it.
 *
 * tt_als_sweep_exact: one outer iteration of Algorithm 1 with every sketched
 * subproblem replaced by the exact one (S^T S = I): right-to-left
 * orthogonalisation, then for k = 0..d-1 the exact update and (k < d-1) QR +
 * absorb.  In this gauge H_k has orthonormal columns, so H_k^T H_k = I.  The
 * left interface is carried from one core to the next, so a sweep reads X
 * twice.  Advances the sweep index like tt_als_sweep; rel_residual as
 * there. */
tt_status tt_exact_rhs(tt_plan plan, const void* X, const void* const* cores, int32_t k, void* B);
tt_status tt_prox_exact(tt_plan plan, const void* X, void* const* cores, int32_t k, void* G_new);
tt_status tt_als_sweep_exact(tt_plan plan, const void* X, void* const* cores, double* rel_residual);

/* QR step of Algorithm 1's inner loop for k < d-1: [Q,R] = qr(G_k^L) by FP64
 * Householder with diag(R) >= 0; G_k <- Q; G_{k+1} <- R G_{k+1}^R.  In place
 * on the device cores (host array of d device pointers). */
tt_status tt_left_orth_absorb(tt_plan plan, void* const* cores, int32_t k);

/* Right-to-left orthogonalisation (Algorithm 1, first step of each outer
 * iteration): for k = d-1..1, LQ of G_k^R via Householder QR of its
 * transpose, G_k <- Q^T, G_{k-1}^L <- G_{k-1}^L R^T.  In place, FP64. */
tt_status tt_right_orthogonalize(tt_plan plan, void* const* cores);

/* Relative residual ||X - [[G]]||_F / ||X||_F (objective (lrtt), Sec. 3),
 * reconstructing the TT on the fly and accumulating in FP64.  Synchronises;
 * *rel_residual receives the value.  Returns TT_ERR_NONFINITE on NaN/Inf. */
tt_status tt_residual(tt_plan plan, const void* X, const void* const* cores, double* rel_residual);

/* Relative change of the cores between two iterates, the accuracy measure
 * the experiments of Sec. 5 stop on: max over k of
 * ||cur_k - prev_k||_F / ||cur_k||_F, summed in FP64.  prev, cur: d device
 * pointers each to FP64 cores of the plan's shapes (the layout of
 * tt_als_sweep); the caller keeps the previous iterate.  Synchronises;
 * *change receives the value.  TT_ERR_NONFINITE (value still written) when
 * some cur_k is zero or a core holds NaN/Inf. */
tt_status tt_core_change(tt_plan plan, const void* const* prev, const void* const* cur, double* change);

/* One outer iteration of Algorithm 1 with the plan's current tables:
 * right-to-left orthogonalisation; then for k = 0..d-1 the interface sketch,
 * the data sketch, the proximal update and (k < d-1) QR + absorb.  Cores are
 * updated in place.  Afterwards the sweep index advances by one and, unless
 * tables were overridden, the next sweep's tables are generated.  If
 * rel_residual is not NULL the residual is computed and the call
 * synchronises. */
tt_status tt_als_sweep(tt_plan plan, const void* X, void* const* cores, double* rel_residual);

/* Schedule of an overlapped sweep (flags without TT_FLAG_SERIAL).  The d data
 * sketches of a sweep depend only on X and the sweep's tables, so they run on
 * a plan-owned side stream while the core updates run on a second plan-owned
 * stream; both fork from and join back into the plan's stream, so the call
 * stays asynchronous and ordered with respect to it.  reserved_cus CUs are
 * left out of the side stream's CU mask (hipExtStreamCreateWithCUMask) for
 * the short kernels of the core updates; 0 gives the side stream every CU.
 * The default (before any call) reserves the CUs of one XCD (CU count / 8;
 * the runtime numbers CUs XCD by XCD), which keeps the two streams on
 * separate L2s, except when the k = 0 pass writes both intermediates
 * (tt_plan_sketch_sources gives 0 for every mode): the core updates then
 * wait for that pass anyway, and no CU is reserved.  TT_ERR_ARG if
 * reserved_cus is negative or not below the
 * device's CU count.  Synchronises and recreates the plan's streams. */
tt_status tt_plan_set_overlap(tt_plan plan, int32_t reserved_cus);

/* Measurement: every launch of the kernels of a timed class below is
 * bracketed by a pair of HIP events recorded on the plan's stream.  Each
 * record leaves a short gap on the GPU (a few microseconds), so time only the
 * classes you need.  Classes: */
#define TT_PROF_SKETCH0 0    /* data sketch main kernel, k = 0 (bucket gather) */
#define TT_PROF_SKETCHK 1    /* data sketch main kernel, k >= 1 (LDS buckets) */
#define TT_PROF_SKETCH_AUX 2 /* data sketch key tables, bucket lists, partial sums, Y_1 from the outer sketch */
#define TT_PROF_INTERFACE 3  /* core CountSketch + FFT, chains, face-split + inverse FFT */
#define TT_PROF_GRAM 4       /* MFMA Gram / right-hand side */
#define TT_PROF_SOLVE 5      /* FP64 partial sums, Cholesky, substitution */
#define TT_PROF_QR 6         /* FP64 Householder QR and absorb */
#define TT_PROF_RESIDUAL 7   /* residual pass */
#define TT_PROF_TABLES 8     /* hash/sign table generation */
#define TT_PROF_EXACT 9      /* exact update: contractions of X with the cores, assembly */
#define TT_PROF_NCLASS 10
#define TT_PROF_ALL 0x3ff    /* every class */
/* enable: bit mask of the classes to time (bit c for class c, TT_PROF_ALL for
 * all of them); 0 stops measurement and releases its events (after
 * synchronising the plan's stream).  Counts already taken are kept until the
 * next read while the mask changes. */
tt_status tt_plan_profile(tt_plan plan, int32_t enable);
/* Synchronise, then return per class the summed milliseconds and the number
 * of launches since the last read (arrays of nclass <= TT_PROF_NCLASS
 * entries, host memory), and reset the counters. */
tt_status tt_plan_profile_read(tt_plan plan, int32_t nclass, double* ms, int64_t* launches);

/* Which data-sketch kernel tt_sketch_tensor runs for mode k of this plan
 * (host query, no device work): TT_SKETCH_PATH_BUCKET for k = 0 (one
 * workgroup per bucket gathers the fibres hashed to it), TT_SKETCH_PATH_STREAM
 * (fibres streamed in memory order into LDS bucket arrays) or
 * TT_SKETCH_PATH_GROUPED (fibres of a column visited in order of their key and
 * summed per key before the LDS scatter) for k >= 1.  TT_ERR_ARG for a bad k
 * or null output. */
#define TT_SKETCH_PATH_BUCKET 0
#define TT_SKETCH_PATH_STREAM 1
#define TT_SKETCH_PATH_GROUPED 2
tt_status tt_plan_sketch_path(tt_plan plan, int32_t k, int32_t* path);

/* Synchronise the plan's stream and report device-side failures recorded so
 * far (TT_ERR_NOT_SPD); clears the recorded status. */
tt_status tt_plan_sync_status(tt_plan plan);

/* Thread-local message describing the last non-OK status ("" if none). */
const char* tt_last_error(void);

/* Library version string. */
const char* tt_version(void);

/* ------------------------------------------------------------------------
 * Learned sketch-size policy.
 *
 * The paper fixes the sketch size only through the bound of Corollary 3
 * (Sec. 4) and notes in Sec. 5 that the bound is conservative.  This
 * extension predicts (log J, log lambda) for each core update from cheap
 * features with a small multilayer perceptron, and falls back to the
 * Corollary 3 bound (capped at the plan's J) when a residual check fails.
 *
 * Network: F = 8 inputs -> 64 -> 64 -> 64 -> 2 outputs, ReLU after each
 * hidden layer, FP32.  Parameters are one device array of
 * TT_JPOLICY_PARAMS floats: for each layer, W (fan_out x fan_in, row-major)
 * then the bias.  Features and targets are row-major B x F and B x 2 device
 * arrays.  Loss: mean over the B x 2 outputs of (y - target)^2.
 * Outputs: y0 = ln J - 7, y1 = log10 lambda + 3.
 * Features of core k at sweep t (tt_jpolicy_features):
 *   ln n_k / 4, ln R_k / 2, ln R_{k+1} / 2, ln(N / n_k) / 16, d / 5, k / d,
 *   t / 10, and the last residual drop log10(res_{t-1} / res_t) (res_{-1} = 1,
 *   0 at t = 0), clipped to [-1, 4].
 * ---------------------------------------------------------------------- */
#define TT_JPOLICY_FEATURES 8
#define TT_JPOLICY_HIDDEN 64
#define TT_JPOLICY_OUTPUTS 2
#define TT_JPOLICY_PARAMS 9026
#define TT_JPOLICY_MAX_BATCH (1 << 20)
/* A predicted J at or above TT_JPOLICY_EXACT_J (three times TT_MAX_J)
 * selects the unsketched update (tt_als_sweep_exact) when the plan has
 * TT_FLAG_EXACT: a sketch that large is no cheaper than the problem itself.
 * Training labels encode that choice as TT_JPOLICY_EXACT_LABEL. */
#define TT_JPOLICY_EXACT_J 24576
#define TT_JPOLICY_EXACT_LABEL 65536
/* tt_jpolicy_choose clamps log10 lambda to the range of the training labels */
#define TT_JPOLICY_LOG10_LAMBDA_MIN (-4.0)
#define TT_JPOLICY_LOG10_LAMBDA_MAX (-1.0)

/* y = net(feats) for B samples (1 <= B <= TT_JPOLICY_MAX_BATCH); device
 * pointers; asynchronous on `stream`. */
tt_status tt_jpolicy_forward(const float* params, const float* feats, int32_t B, float* out, void* stream);

/* Gradient of the loss w.r.t. the parameters (TT_JPOLICY_PARAMS floats,
 * overwritten) and the loss itself (one float), for B samples
 * (1 <= B <= 4096), by backpropagation in one workgroup with a fixed
 * summation order (deterministic).  Device pointers; asynchronous. */
tt_status tt_jpolicy_loss_grad(const float* params, const float* feats, const float* targets, int32_t B, float* grad,
                               float* loss, void* stream);

/* One Adam step (Kingma and Ba) on `count` parameters in place, step >= 1
 * (bias corrections 1 - beta^step).  m, v: device moment arrays of the same
 * length, updated in place.  Asynchronous. */
tt_status tt_jpolicy_adam(float* params, float* m, float* v, const float* grad, int64_t count, int64_t step, float lr,
                          float beta1, float beta2, float eps, void* stream);

/* Features of every core update of the plan at sweep t (host output, d x F
 * floats, row k = core k).  No device work. */
tt_status tt_jpolicy_features(tt_plan plan, int64_t t, double last_drop, float* feats);

/* Apply the network to the plan's d feature rows (in the plan's workspace, on
 * its stream; synchronises) and return the sweep's sketch size and lambda:
 * J = the largest of the d predictions, rounded to the nearest product of
 * 2, 3, 5, 7 in [J_min, plan J], or 0 (the unsketched update) when that
 * prediction is at least TT_JPOLICY_EXACT_J and the plan has TT_FLAG_EXACT;
 * lambda = the prediction of that core, clamped to
 * [10^TT_JPOLICY_LOG10_LAMBDA_MIN, 10^TT_JPOLICY_LOG10_LAMBDA_MAX]. */
tt_status tt_jpolicy_choose(tt_plan plan, const float* params, int64_t t, double last_drop, int64_t J_min, int64_t* J,
                            double* lambda);

/* Corollary 3 (Sec. 4): m = max{8 s^2 (2 + 3^q) / delta, 8 s (2 + 3^q) /
 * (eps delta)} for s unknowns per column and q sketched modes.
 * TT_ERR_ARG unless s >= 1, q >= 1, 0 < eps, 0 < delta < 1. */
tt_status tt_sketch_size_bound(int64_t s, int32_t q, double eps, double delta, double* m);

/* Fallback sketch size of the plan: the largest Corollary 3 bound over its
 * core updates (s = R_k R_{k+1}, q = d - 1), capped at the plan's J and
 * rounded down to a product of 2, 3, 5, 7. */
tt_status tt_plan_fallback_J(tt_plan plan, double eps, double delta, int64_t* J);

/* Run sweeps until the exact relative residual is <= target or max_sweeps
 * sweeps are done.  With params == NULL every sweep uses the plan's current
 * J and lambda.  Otherwise the policy chooses (J, lambda) before each sweep
 * from the features above, J = 0 meaning an exact sweep (tt_als_sweep_exact)
 * with the chosen lambda; when a sweep (from the second on) does not lower
 * the previous sweep's residual, the next sweep is the fallback: an exact
 * sweep (tt_als_sweep_exact, recorded with J = 0) when the plan has
 * TT_FLAG_EXACT and the Corollary 3 size (eps = 0.5, delta = 0.1) of some
 * core update is at least its N / n_k (a sketch no smaller than the
 * problem), else a sketched sweep at tt_plan_fallback_J; both with the
 * descriptor's lambda.  The residual of every sweep is computed exactly and
 * read back (synchronising).  residuals, Js, lambdas: host arrays of
 * max_sweeps entries or NULL. */
typedef struct {
  int32_t sweeps;      /* sweeps performed */
  int32_t reached;     /* 1 if the last residual <= target */
  int32_t fallbacks;   /* sweeps run at the fallback size */
  double residual;     /* last exact relative residual */
} tt_run_stats;
tt_status tt_als_run(tt_plan plan, const void* X, void* const* cores, const float* params, int32_t max_sweeps,
                     double target, int64_t J_min, double* residuals, int64_t* Js, double* lambdas,
                     tt_run_stats* stats);

/* ------------------------------------------------------------------------
 * Batched form: many independent problems of uneven shapes and ranks advance
 * together.  Each problem is described by its own tt_plan_desc (FP32 X, FP32
 * work, TT_GRAM_WORK; n_0 <= 256; any order, ranks, J, lambda, seed).  A
 * sweep runs step k = 0, 1, ... for all problems of order > k: the interface
 * sketches and core updates of all of them (one launch per kernel), and ONE
 * persistent data-sketch launch covering every participating problem.  The whole sweep can be captured into
 * a hipGraph (tt_batch_set_graph) and replayed; tables then follow a device
 * sweep counter.  The batch owns one plan per problem; all device memory is
 * one caller workspace.
 * ---------------------------------------------------------------------- */
#define TT_BATCH_MAX 4096
typedef struct tt_batch_s* tt_batch;

/* descs: count descriptors (host).  Reports the workspace size. */
tt_status tt_batch_plan(int32_t count, const tt_plan_desc* descs, void* hip_stream, size_t* workspace_bytes,
                        tt_batch* out);
tt_status tt_batch_bind_workspace(tt_batch batch, void* dev_workspace, size_t bytes);
tt_status tt_batch_destroy(tt_batch batch);

/* The plan of problem i, owned by the batch (for queries such as
 * tt_plan_get_tables; do not destroy it, rebind it or change its sweep). */
tt_status tt_batch_get_plan(tt_batch batch, int32_t i, tt_plan* plan);

/* Capture sweeps into a hipGraph (enable = 1) or enqueue them directly (0).
 * A graph is re-captured when the X or core pointers change. */
tt_status tt_batch_set_graph(tt_batch batch, int32_t enable);

/* The batched data sketch of step k alone: Y[i] (J_i x n_k, column-major,
 * FP32, device) for every problem of order > k; Y[i] of the others is not
 * touched.  X: count device pointers.  Problems whose plans take Y_1 from
 * the outer sketch of the k = 0 pass (tt_plan_sketch_sources) get it the
 * same way here: their step-0 launch writes that sketch beside Y_0, and
 * step 1 reads it back instead of X, so asking for k = 1 runs step 0 first.
 * Y == NULL runs the launches of step k only (the results stay in the
 * problems' plans; at k = 1 the outer sketch is read as step 0 left it),
 * e.g. to time them. */
tt_status tt_batch_sketch_tensor(tt_batch batch, const void* const* X, int32_t k, void* const* Y);

/* Which data-sketch kernel the batched launch of step k runs (host query, no
 * device work): TT_BSKETCH_PATH_BUCKET for k = 0 (one workgroup per (problem,
 * bucket) gathers the fibres hashed to it), TT_BSKETCH_PATH_FIBRES (mode-0
 * fibres streamed into LDS bucket arrays; k = 1, and k >= 2 when slabs do not
 * fit in LDS), TT_BSKETCH_PATH_SLABS (for k >= 2, the contiguous n_0 x n_1
 * slabs streamed 64 entries at a time with a per-problem LDS key table) or
 * TT_BSKETCH_PATH_SLABS_SORTED (the same slabs read whole in the order of a
 * per-step key sort, slabs of one key summed in registers), as the step's
 * current tuning selects.  TT_ERR_ARG for k outside [0, max order) or null
 * output. */
#define TT_BSKETCH_PATH_BUCKET 0
#define TT_BSKETCH_PATH_FIBRES 1
#define TT_BSKETCH_PATH_SLABS 2
#define TT_BSKETCH_PATH_SLABS_SORTED 3
tt_status tt_batch_sketch_path(tt_batch batch, int32_t k, int32_t* path);

/* One sweep of every problem.  X: count device pointers; cores: count host
 * arrays of d_i device core pointers.  residuals: NULL, or count host doubles
 * receiving each problem's exact relative residual (synchronises). */
tt_status tt_batch_sweep(tt_batch batch, const void* const* X, void* const* const* cores, double* residuals);

/* Autotuner: for every step, time (reps launches each, after one warm-up)
 * and keep the fastest of
 *  - the data-sketch launch over its shapes: entries of a fibre per lane
 *    (2 when every n_0 <= 128, or 4), fibres per lane group in flight (4 or 8
 *    at k = 0, 8 or 16 at k >= 1), and for k >= 1 workgroup counts of 1/2,
 *    1, 2, 4 and 8 times the device occupancy of that shape (at most 16384);
 *    slab steps (k >= 2 when the slabs fit in LDS) take 4 or 8 in that
 *    field for the stream of 64-entry rows in memory order (rows per lane in
 *    flight), or 1 or 2 for the key-sorted slab stream (each column's slabs
 *    sorted by their key over the modes other than 0, 1 and k, read whole,
 *    slabs of one key summed in registers; slabs per lane group in flight;
 *    offered when every problem's N / (n_0 n_1) is below 2^31); the entries
 *    per lane stay as set;
 *  - the Gram K-chunk of the step's core updates (256, 512 or 1024 rows of SH
 *    per partial product), timed with the partial sums.
 * The choices stay with the batch (tt_batch_get_tuning exports them for a
 * caller to keep, tt_batch_set_tuning restores them).  chosen: NULL or host
 * int64 array of max order entries receiving the workgroup count per step
 * (0 for k = 0).  Drops a captured graph. */
tt_status tt_batch_autotune(tt_batch batch, const void* const* X, int32_t reps, int64_t* chosen);

/* The batch's tuning, TT_MAX_ORDER steps of TT_BATCH_TUNE_FIELDS int64:
 * [0] workgroups of the data-sketch launch (0: device occupancy; 0 at k = 0),
 * [1] entries per lane, [2] fibres (slab steps: rows, or for the key-sorted
 * slab stream slabs) per lane group in flight, [3] Gram K-chunk.  set validates every used step (values as listed under
 * tt_batch_autotune; the K-chunk may be any multiple of 256 up to 8192) and
 * returns TT_ERR_ARG, changing nothing, on the first bad one; it drops a
 * captured graph.  Steps at or beyond the largest order are ignored. */
#define TT_BATCH_TUNE_FIELDS 4
tt_status tt_batch_get_tuning(tt_batch batch, int64_t* tuning);
tt_status tt_batch_set_tuning(tt_batch batch, const int64_t* tuning);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under stream capture,
 * serving loops and harnesses that forbid hipMalloc): tt_residual without a
 * plan or a workspace.
 *
 * Computes ||X - [[G]]||_F / ||X||_F exactly as tt_residual does (same
 * kernels, same launch shape, so the same value) for the tensor described by
 * d, n (d mode sizes) and r (d + 1 ranks, r[0] = r[d] = 1, each <= TT_MAX_RANK)
 * with X in x_dtype and the sums in work_dtype (TT_F64 or TT_F32).  X and the
 * d FP64 cores (host array of device pointers, core k of shape
 * (r[k], n[k], r[k+1]), first index fastest) are device memory owned by the
 * caller; n, r and cores are read during the call only.  Work is enqueued on
 * hip_stream (a hipStream_t of the current device, NULL for the null stream)
 * and the call synchronises it to read the result.
 *
 * Scratch: the per-wave partials, u(o) (prod n[2..d-1] x r[2] work-type
 * values) and, when room is left, G_0 x G_1 (n[0] n[1] x r[2]) sit in one
 * static device array of TT_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends.  The call allocates nothing: no hipMalloc, hipFree or
 * allocating library call.  Every call on a GPU uses that GPU's array, so
 * calls that overlap on one GPU (other streams, other host threads) race:
 * serialise them.  Errors: TT_ERR_ARG / TT_ERR_SHAPE (including a scratch
 * need above TT_NOALLOC_SCRATCH_BYTES) before any device work; TT_ERR_HIP;
 * TT_ERR_NONFINITE for a NaN or Inf residual. */
#define TT_NOALLOC_SCRATCH_BYTES (32 << 20)
tt_status tt_residual_noalloc(int32_t d, const int64_t* n, const int64_t* r, tt_dtype x_dtype, tt_dtype work_dtype,
                              const void* X, const void* const* cores, void* hip_stream, double* rel_residual);

#ifdef __cplusplus
}
#endif

#endif /* TT_SKETCH_H */
