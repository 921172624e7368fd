/*
 * srm.h -- C-ABI of the MI355X (gfx950) Shared Response Model EM library.
 *
 * The library fits the probabilistic Shared Response Model (SRM) of
 * arXiv 1608.04647, Sec. II, with the distributed EM of Algorithm 1 (D-SRM):
 *
 *   model (Sec. II-A, Eq. 1):  x_it = W_i s_t + mu_i + eps_i,
 *                              eps_i ~ N(0, rho_i^2 I), s_t ~ N(0, Sigma_s),
 *                              W_i^T W_i = I,
 *   E-step (Eq. 7-10):         Y = sum_i rho_i^-2 W_i^T Xhat_i,
 *                              M = (Sigma_s^-1 + rho0 I)^-1, rho0 = sum rho_i^-2,
 *                              S = E[S] = Sigma_s [I - rho0 M] Y,
 *   M-step (Eq. 4, 5, 11):     Sigma_s = M + S S^T / t,
 *                              A_i = Xhat_i S^T, W_i = A_i (A_i^T A_i)^-1/2,
 *                              rho_i^2 = (||Xhat_i||^2 - 2 tr(W_i^T A_i)
 *                                         + t tr(Sigma_s)) / (t v_i).
 *
 * The rho_i^2 update is the exact maximiser of the expected complete-data
 * log-likelihood; the printed Eq. 5 is garbled (a missing 1/(T V) factor and
 * the total V where v_i belongs).  The factor 1/2 printed in A_i is dropped
 * (the polar factor is scale invariant).  Sigma_s starts at I, rho_i^2 at 1,
 * and W_i at the caller's orthonormal W0_i or a seeded random orthonormal map
 * the library draws (srm_init).  The log-likelihood reported per
 * iteration is the marginal Gaussian log-density of the demeaned data under
 * the parameters entering that iteration, reduced with the inversion lemma
 * (Eq. 7) and Eq. 8.
 *
 * Conventions shared by every entry point:
 *  - Every function returns srm_status; no C++ exception crosses the ABI.
 *    On failure, srm_last_error() returns a message (per thread).
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary process memory.
 *  - The library never allocates device memory: everything it keeps lives in
 *    the caller's workspace (see srm_workspace_size), which must stay valid
 *    and untouched until srm_free().  The one exception is the static 8 MiB
 *    array of srm_transform_static, part of the library image on each device.
 *  - All device work is enqueued on desc.hip_stream (a hipStream_t; NULL means
 *    the library creates its own non-blocking stream).  Calls that return host
 *    values synchronise that stream; the others only enqueue.
 *  - Matrices are row-major.  X_i is v_i x t (voxels x TRs) with row stride t.
 *  - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef SRM_H_
#define SRM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srm_ctx srm_ctx; /* opaque; owned by the library */

typedef enum {
  SRM_OK = 0,
  SRM_E_ARG = 1,       /* invalid argument (sizes, NULL pointers, precision)   */
  SRM_E_WORKSPACE = 2, /* workspace NULL, misaligned or smaller than required */
  SRM_E_HIP = 3,       /* a HIP runtime call failed                            */
  SRM_E_RANK = 4,      /* A_i^T A_i numerically singular: lambda_min <= 1e-13 lambda_max */
  SRM_E_NOTPD = 5,     /* Sigma_s or Sigma_s^-1 + rho0 I not positive definite */
  SRM_E_NONFINITE = 6, /* NaN or Inf in the input data                         */
  SRM_E_STATE = 7      /* call not valid in the context's current state        */
} srm_status;

/* Storage format of the demeaned data Xhat_i inside the workspace.
 * SRM_FP32:   float32, FP32 matrix-core products.
 * SRM_BF16:   one bfloat16 per element; W_i and S enter as bf16 hi+lo pairs
 *             (2 bf16 products per multiply, FP32 accumulation).
 * SRM_BF16X2: Xhat_i = hi + lo, both bfloat16 (3 bf16 products per multiply,
 *             the lo*lo term dropped, FP32 accumulation).
 * The k x k steps (Cholesky, Jacobi eigensolver, polar factor, rho_i^2) and
 * the cross-subject reductions run in FP64 in every format.               */
typedef enum { SRM_FP32 = 0, SRM_BF16 = 1, SRM_BF16X2 = 2 } srm_prec;

enum {
  SRM_NO_GRAPH = 1u,    /* launch each iteration's kernels directly instead of
                           replaying one captured hipGraph                     */
  SRM_NO_W0_CHECK = 2u, /* skip the host check that W0_i^T W0_i = I            */
  SRM_TWO_PASS = 4u,    /* use the two-pass sweep (A = Xhat S^T to HBM, then
                           A^T Xhat) even where the fused one-pass sweep applies
                           (BF16 forms with k <= 64 and t <= 512)              */
  SRM_X_HOST = 8u,      /* the X[i] of srm_init and X_i of srm_ingest are host
                           pointers: each subject is uploaded in chunks through
                           two staging buffers in the workspace on a second
                           stream and converted there (no full FP32 copy on
                           the device)                                        */
  SRM_ZSCORE = 16u,     /* standardise each voxel (the z-score preprocessing of
                           the paper's implementation, Sec. IV-A): after the
                           mean, divide by the population standard deviation
                           over the t samples (1/t).  A constant voxel is only
                           demeaned.  srm_transform and srm_map apply the same
                           per-voxel scale.                                    */
  SRM_GRAM = 32u,       /* sample-space iteration (the Discussion's change of
                           complexity from voxels to samples): srm_init forms
                           G_i = Xhat_i^T Xhat_i (t x t; FP32 for the BF16
                           forms, FP64 for SRM_FP32 storage: N t^2 4 or 8 bytes
                           of workspace) in one pass over the data; each iteration
                           then uses A_i^T Xhat_i = S G_i and A_i^T A_i =
                           S G_i S^T and reads no voxel data.  The same EM
                           iterate as the streamed sweep up to rounding; pays
                           off when t is well below the voxel counts.  At most
                           65535 subjects.                                    */
  SRM_AUTOTUNE = 64u    /* srm_init_end picks the sweep's launch shapes
                           (srm_tuning) for this problem and device: from the
                           on-disk cache ($SRM_TUNE_CACHE, else
                           $HOME/.cache/srm_tune.tsv; an empty SRM_TUNE_CACHE
                           disables it), else by srm_autotune with 2 timed
                           iterations per shape, whose result is appended to
                           the cache.  Without it the default shapes are used. */
};

typedef struct {
  int32_t n_subjects;   /* N >= 1                                              */
  const int64_t *v;     /* host [N]: voxels per subject, k <= v_i < 2^31       */
  int64_t t;            /* TRs (samples), 2 <= t <= 65536, k <= t              */
  int32_t k;            /* shared features, 1 <= k <= 128                      */
  srm_prec prec;        /* storage format of Xhat                              */
  uint32_t flags;       /* SRM_* flags above                                   */
  void *hip_stream;     /* hipStream_t or NULL                                 */
} srm_desc;

/* Bytes of device workspace srm_init needs for this problem (Sec. II-C, II-D:
 * the E-step keeps only k x k and k x t state beside the data).  Returns
 * SRM_E_ARG for an invalid descriptor. */
srm_status srm_workspace_size(const srm_desc *desc, size_t *bytes);

/* Algorithm 1, initialisation: demean each X_i (mu_i = row means over t),
 * store Xhat_i in desc->prec inside the workspace, compute c_i = ||Xhat_i||^2
 * from the stored values, set the starting maps W_i, rho_i^2 = 1,
 * Sigma_s = I, and run the first E-step (its log-likelihood is the first one
 * srm_fit reports).  Equivalent to srm_init_begin, srm_ingest of every
 * subject in order, and srm_init_end.
 *   X:  host array of N device pointers (host pointers with SRM_X_HOST);
 *       X[i] is v_i x t float32, row stride t.  Read during the call only
 *       (the caller keeps ownership).
 *   W0: NULL, or a host array of N host pointers; W0[i] is v_i x k float64
 *       with orthonormal columns (checked: max|W0^T W0 - I| <= 1e-8 unless
 *       SRM_NO_W0_CHECK), read during the call only.  Where W0 or W0[i] is
 *       NULL the library draws subject i's start itself: Algorithm 1's random
 *       orthonormal start, taken as the polar factor G (G^T G)^-1/2 of a
 *       v_i x k matrix G of N(0, 1) entries, which is Haar distributed.  Entry
 *       e = r k + c of G is normal number e % 4 of the Philox4x64-10 block
 *       (Salmon et al., SC 2011) with counter (e / 4, i, 0, 0) and key
 *       (seed, 0), by the Box-Muller transform of the block's 64-bit words
 *       x taken as u = (floor(x / 2^11) + 1/2) 2^-53: words 0, 1 give
 *       sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1), words 2, 3 likewise.
 *   seed: Philox key word 0 for the drawn starts (unused when every W0[i]
 *       is given).
 *   workspace: device memory of at least srm_workspace_size bytes, 256-byte
 *       aligned, owned by the caller, used exclusively by this context.
 * Errors: SRM_E_ARG, SRM_E_WORKSPACE, SRM_E_NONFINITE, SRM_E_HIP, SRM_E_NOTPD,
 * SRM_E_RANK (a drawn start or a W0 whose polar factor does not exist).
 * On success *out is a new context (free with srm_free); on failure none. */
srm_status srm_init(srm_ctx **out, const srm_desc *desc, const float *const *X,
                    const double *const *W0, uint64_t seed, void *workspace,
                    size_t ws_bytes);

/* Incremental initialisation, for data that should not be held in memory all
 * at once (the per-subject loading of the paper's implementation, Sec. IV-B).
 *  srm_init_begin: validates the descriptor and workspace and returns a
 *      context awaiting its subjects (the same arguments as srm_init, without
 *      the data).  Only srm_ingest, srm_init_end, srm_get_info and srm_free
 *      are valid on it until srm_init_end succeeds (SRM_E_STATE otherwise).
 *  srm_ingest: demeans, converts and stores subject i (any order, once each).
 *      X_i: v_i x t float32, row stride t; a device pointer, or a host pointer
 *      with SRM_X_HOST, in which case the rows are uploaded in chunks through
 *      two staging buffers of the workspace on a second stream, each chunk's
 *      upload overlapping the conversion of the previous one.  W0_i: v_i x k
 *      float64 host map with orthonormal columns, or NULL to draw subject i's
 *      start as described under srm_init.  Both are read during the call only:
 *      the caller may free or reuse them when it returns.
 *      Errors: SRM_E_ARG (index, NULL X_i, repeated subject, W0_i not
 *      orthonormal), SRM_E_STATE (after srm_init_end), SRM_E_HIP.  A failed
 *      call leaves subject i not ingested.
 *  srm_init_end: checks that every subject was ingested (SRM_E_STATE
 *      otherwise), rejects NaN or Inf data (SRM_E_NONFINITE), forms G_i with
 *      SRM_GRAM, and runs the first E-step (SRM_E_RANK, SRM_E_NOTPD).  On any
 *      failure the context stays unusable and must be freed. */
srm_status srm_init_begin(srm_ctx **out, const srm_desc *desc, uint64_t seed,
                          void *workspace, size_t ws_bytes);
srm_status srm_ingest(srm_ctx *ctx, int32_t i, const float *X_i, const double *W0_i);
srm_status srm_init_end(srm_ctx *ctx);

/* One EM iteration of Algorithm 1 (M-step on the current posterior, then the
 * next E-step).  loglik (host, nullable) receives the log-likelihood of the
 * parameters entering the iteration.  Synchronises the stream.
 * Errors as srm_fit. */
srm_status srm_em_step(srm_ctx *ctx, double *loglik);

/* n_iter >= 0 EM iterations (fixed count; the paper's stopping criterion is
 * unspecified).  loglik (host [n_iter], nullable) receives the log-likelihood
 * of the parameters entering each iteration.  The iterations are enqueued
 * without host synchronisation (one captured hipGraph replayed per iteration
 * unless SRM_NO_GRAPH; srm_get_info says which ran); the stream is
 * synchronised once at the end.
 * Errors: SRM_E_RANK (some A_i^T A_i numerically singular, reading of the
 * polar factor's existence), SRM_E_NOTPD, SRM_E_HIP, SRM_E_STATE.  On
 * SRM_E_RANK or SRM_E_NOTPD the iteration that failed and every later one in
 * the call stop at their first kernel, and the carried state (everything
 * srm_get_state returns, the iteration count included) is put back to what
 * it was when the call started. */
srm_status srm_fit(srm_ctx *ctx, int32_t n_iter, double *loglik);

/* Kernel phases of one iteration, in launch order (indices of srm_profile):
 *  SRM_PHASE_MPHASE    A = Xhat S^T over all subjects (Eq. 4, A_i)
 *  SRM_PHASE_EPHASE    per-slice A^T Xhat and A^T A (Eq. 10 partials, Eq. 4 Gram)
 *  SRM_PHASE_POLAR     per-subject FP64 polar factor (Newton-Schulz from the
 *                      previous one or from G_i / |G_i|_F, else Jacobi) and
 *                      rho_i^2 (Eq. 4-5)
 *  SRM_PHASE_EREDUCE   Y = sum_i rho_i^-2 W_i^T Xhat_i (Eq. 10 reduction)
 *  SRM_PHASE_POSTERIOR k x k posterior, S, Sigma_s, log-likelihood (Eq. 7-11)
 *  SRM_PHASE_FUSED     one-pass sweep forming A, A^T Xhat and A^T A together
 *  SRM_PHASE_GRAM      sample-space products S G_i and S G_i S^T (SRM_GRAM)
 *                      (replaces MPHASE + EPHASE where it applies) */
enum {
  SRM_PHASE_MPHASE = 0,
  SRM_PHASE_EPHASE = 1,
  SRM_PHASE_POLAR = 2,
  SRM_PHASE_EREDUCE = 3,
  SRM_PHASE_POSTERIOR = 4,
  SRM_PHASE_FUSED = 5,
  SRM_PHASE_GRAM = 6,
  SRM_NPHASE = 7
};

/* Runs n_iter iterations like srm_fit but with direct kernel launches, each
 * kernel bracketed by HIP events on the context's stream, and adds each
 * phase's measured milliseconds into ms[SRM_NPHASE] (host; zeroed first).
 * Synchronises after every iteration; meant for measurement, not speed.
 * Errors and their undoing as srm_fit. */
srm_status srm_profile(srm_ctx *ctx, int32_t n_iter, double *ms);

/* Project new samples of subject i into the shared space (Sec. II-A:
 * s = W_i^T (x - mu_i)):  S_out = W_i^T (X_new - mu_i 1^T).
 *   X_new: device, v_i x t_new float32, row stride t_new (t_new >= 1).
 *   S_out: device, k x t_new float32, row stride t_new.
 * Valid after at least one iteration (SRM_E_STATE otherwise).  Enqueues only. */
srm_status srm_transform(srm_ctx *ctx, int32_t i, const float *X_new,
                         int64_t t_new, float *S_out);

/* srm_transform for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * S_out = W_i^T (X_new - mu_i 1^T) with the same arguments, in one launch
 * pair over all t_new columns, its partial sums held in a static device
 * array of 8 MiB that the library keeps on each device it runs on until the
 * process ends (no allocation of any kind in the call).  Every call on one
 * device shares that array: calls that overlap on one device (from any
 * context or stream) race and must be serialised by the caller.
 * Errors as srm_transform, plus SRM_E_ARG when one row split of t_new
 * columns exceeds the array (t_new > 2^21 / k_padded, k_padded = k rounded up
 * to 16) and SRM_E_HIP when the array's address could not be obtained at
 * srm_init_begin.  Enqueues only. */
srm_status srm_transform_static(srm_ctx *ctx, int32_t i, const float *X_new,
                                int64_t t_new, float *S_out);

/* Map new samples of subject i into subject j's voxel space through the
 * shared space (Sec. II-A): Y_out = W_j W_i^T (X_new - mu_i 1^T), i.e. the
 * projection of srm_transform followed by W_j.  The result is in subject j's
 * demeaned space (add mu_j, from srm_get_mu, for its raw space).
 *   X_new: device, v_i x t_new float32, row stride t_new.
 *   Y_out: device, v_j x t_new float32, row stride t_new.
 * Valid after at least one iteration (SRM_E_STATE otherwise).  Enqueues only. */
srm_status srm_map(srm_ctx *ctx, int32_t i, int32_t j, const float *X_new,
                   int64_t t_new, float *Y_out);

/* Results of the last completed iteration (SRM_E_STATE before the first).
 *  srm_get_w:      device dst, v_i x k float32: W_i (orthonormal columns).
 *  srm_get_s:      device dst, k x t float32: the shared response E[S] of the
 *                  E-step the final W_i were built from.
 *  srm_get_rho2:   host dst [N] float64.
 *  srm_get_sigma_s:host dst k x k float64.
 *  srm_get_mu:     device dst, v_i float64: subject i's voxel means.
 *  srm_get_scale:  device dst, v_i float64: the per-voxel factor applied after
 *                  demeaning (1/std with SRM_ZSCORE, else 1).  Valid from
 *                  srm_init on, like srm_get_mu.
 *  srm_get_loglik: host dst [capacity] float64, all log-likelihoods computed so
 *                  far (n_iter + 1 after n_iter iterations: the last one is the
 *                  log-likelihood of the final parameters); *count receives
 *                  their number (dst may be NULL to query it).
 * The host getters synchronise the stream. */
srm_status srm_get_w(srm_ctx *ctx, int32_t i, float *dst);
srm_status srm_get_s(srm_ctx *ctx, float *dst);
srm_status srm_get_rho2(srm_ctx *ctx, double *dst);
srm_status srm_get_sigma_s(srm_ctx *ctx, double *dst);
srm_status srm_get_mu(srm_ctx *ctx, int32_t i, double *dst);
srm_status srm_get_scale(srm_ctx *ctx, int32_t i, double *dst);
srm_status srm_get_loglik(srm_ctx *ctx, double *dst, int32_t capacity,
                          int32_t *count);

/* Checkpoint and resume.  The state between iterations is the posterior of
 * the last E-step (S, Sigma_s, tr Sigma_s, the k x k matrices M), the
 * per-subject rho_i^2 and polar factors P_i with their eigenvectors, the
 * log-likelihood history and the iteration count (Algorithm 1 carries exactly
 * these from one iteration to the next; the data enter through Xhat_i only).
 *  srm_get_state: host blob; with blob == NULL, *bytes receives the size.
 *                 Otherwise *bytes must hold at least that size.  Valid from
 *                 srm_init_end on (a blob taken before the first iteration
 *                 resumes from the first E-step).  Synchronises the stream.
 *  srm_set_state: host blob from srm_get_state of a context with the same
 *                 descriptor (N, v, t, k, format, sweep) and the same data
 *                 (checked through c_i = ||Xhat_i||_F^2, bitwise): SRM_E_ARG
 *                 otherwise.  Continuing from a restored state gives results
 *                 bitwise identical to an uninterrupted fit.  Synchronises. */
srm_status srm_get_state(srm_ctx *ctx, void *blob, size_t *bytes);
srm_status srm_set_state(srm_ctx *ctx, const void *blob, size_t bytes);

/* Number of completed iterations. */
srm_status srm_iterations(const srm_ctx *ctx, int32_t *n);

/* How the context runs its iterations (no device work; valid from
 * srm_init_begin on). */
enum {
  SRM_SWEEP_ONE_PASS = 0, /* A = Xhat S^T, A^T Xhat and A^T A in one pass over Xhat */
  SRM_SWEEP_TWO_PASS = 1, /* A to HBM, then A^T Xhat and A^T A              */
  SRM_SWEEP_GRAM = 2      /* sample-space products on G_i (SRM_GRAM)         */
};
typedef struct {
  int32_t sweep;          /* SRM_SWEEP_*                                          */
  int32_t graph;          /* 1: the last srm_fit replayed one captured hipGraph
                             per iteration; 0: direct launches (SRM_NO_GRAPH, a
                             failed capture, or no srm_fit yet)                */
  int32_t k_padded;       /* k rounded up to the matrix-core tile (16)           */
  int32_t n_ranges;       /* workgroups of the streaming sweep (equal row ranges) */
  int32_t n_slices;       /* row ranges split at subject boundaries              */
  int32_t reserved[3];
  int64_t ldt;            /* stored row stride of Xhat (t padded)               */
  size_t workspace_bytes; /* = srm_workspace_size                                */
} srm_info;
srm_status srm_get_info(const srm_ctx *ctx, srm_info *info);

/* Launch shapes of the sweep.  Every candidate computes the same EM iterate
 * (Algorithm 1); they differ in how the work is cut into workgroups and so
 * in the order of the FP32 partial sums, hence in rounding (results are
 * bitwise reproducible for a given shape).
 *  sweep_kernel   one-pass sweep only: SRM_KERNEL_RING (Xhat streamed from
 *                 HBM through a register ring, read again from the caches by
 *                 the second half) or SRM_KERNEL_STAGED (each 32-row chunk
 *                 of Xhat loaded once into LDS and both halves read it
 *                 there; K padding 16 or 32, 48 with t in (256, 384], 64 with t in
 *                 (128, 256] or (384, 512])
 *  sweep_wgs      workgroups (equal row ranges) of the streaming sweep:
 *                 256, 512, 768, 1024 (one-pass) or 256, 512, 1024 (two-pass)
 *  chunk_rows     rows per chunk of the one-pass sweep (ring: 64, or 16 x
 *                 the 64-TR column panels; staged: 32); 0 otherwise
 *  reduce_wgs     workgroups of the E-step reduction: 256, 512 or 1024
 *  mphase_rounds  two-pass sweep: residency rounds of M-phase row tiles (1, 2);
 *                 0 otherwise
 * srm_get_tuning: the shapes in use (valid from srm_init_begin on).
 * srm_set_tuning: puts one of srm_tuning_candidates in place (SRM_E_ARG for
 *                 anything else); valid between iterations.
 * srm_tuning_candidates: all candidates for this problem (out may be NULL to
 *                 query *count; at most capacity are written).
 * srm_autotune:   times candidates (one warm-up and `trials` iterations each,
 *                 direct launches, HIP events around the phases the shapes
 *                 change: the sweep kernels, the E-step reduction and the
 *                 posterior, which reads one reduction partial per subject
 *                 group; not the polar step) by coordinate search (the sweep's
 *                 shapes, then the reduction's), starting from the shapes in
 *                 use, which a candidate replaces only when it is more than 1%
 *                 faster; restores the carried state after every trial, puts
 *                 the fastest in place, appends it to the cache and returns it
 *                 (best, and best_ms, those phases' milliseconds per
 *                 iteration; both nullable).  A numeric failure in a trial
 *                 returns its status with the state and shapes unchanged. */
enum { SRM_KERNEL_RING = 0, SRM_KERNEL_STAGED = 1 };
typedef struct {
  int32_t sweep_kernel;
  int32_t sweep_wgs;
  int32_t chunk_rows;
  int32_t reduce_wgs;
  int32_t mphase_rounds;
  int32_t reserved[3];
} srm_tuning;
srm_status srm_get_tuning(const srm_ctx *ctx, srm_tuning *t);
srm_status srm_set_tuning(srm_ctx *ctx, const srm_tuning *t);
srm_status srm_tuning_candidates(const srm_ctx *ctx, srm_tuning *out, int32_t capacity,
                                 int32_t *count);
srm_status srm_autotune(srm_ctx *ctx, int32_t trials, srm_tuning *best, double *best_ms);

/* Message for the last failed call on this thread ("" if none). */
const char *srm_last_error(void);

/* Frees the context (not the caller's workspace).  NULL is ignored. */
void srm_free(srm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SRM_H_ */
