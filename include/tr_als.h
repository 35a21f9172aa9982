/*
 * tr_als.h -- C ABI of the MI355X (gfx950) tensor-ring ALS library.
 *
 * Method: "Practical Alternating Least Squares for Tensor Ring Decomposition"
 * (Yu & Li, arXiv 2210.11362).  The library runs the mode-n ALS update of
 * Sec. 3 on one GPU:
 *   (a) the MTTSP  M_n = X_[n] G^{!=n}_[2]  (Alg. 2, MTTSP step), streamed from
 *       HBM in one pass with the subchain rows formed in LDS;
 *   (b) the coefficient matrix S_n<2> = (G^{!=n}_[2])^T G^{!=n}_[2] formed from
 *       per-core Gram matrices multiplied around the ring (Prop. 3.1, Alg. 2);
 *   (c) the normal-equation solve G_n(2) S_n<2> = M_n (Alg. 2) with iterative
 *       refinement, or the QR-stabilised update of Alg. 3.
 *
 * Conventions
 *   - Every pointer is a DEVICE pointer unless its comment says "host".
 *   - Layout follows the paper's index rule (Sec. 2): the first index is fastest.
 *     X holds prod(I_n) elements with i_1 fastest.  Core n (R_n x I_n x R_{n+1},
 *     R_{N+1} = R_1) holds element (a, i, b) at offset a + R_n*(i + I_n*b).
 *   - Matrices returned by the introspection calls are column-major FP64.
 *   - Work is enqueued on the caller's hipStream_t (passed as void*; NULL means
 *     the default stream).  A context is used by one host thread at a time;
 *     separate contexts are independent.
 *   - Return value: TR_OK (0) or a negative TR_E* code.  tr_als_last_error()
 *     gives the context's message.  Nothing fails silently: there is no hidden
 *     regularisation and no CPU fallback.
 */
#ifndef TR_ALS_H
#define TR_ALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tr_als_ctx tr_als_ctx;

/* Update variant (Alg. 2 normal equation, Alg. 3 QR, Alg. 4 QR + normal
 * equation). */
enum { TR_NE = 0, TR_QR = 1, TR_QRNE = 2 };

/* Solve of the mode update (tr_als_set_solve). */
enum { TR_SOLVE_FACTOR = 0, TR_SOLVE_PINV = 1 };

/* Element types: storage type of X (TR_F64 or TR_F32) and the precision of the
 * X contraction (all four).  The Gram, ring, solve and QR steps are always FP64. */
enum { TR_F64 = 0, TR_F32 = 1, TR_BF16 = 2, TR_FP8 = 3 };

/* Status codes. */
enum {
  TR_OK = 0,
  TR_EINVAL = -1,      /* bad argument (sizes, ranks, dtype, variant, NULL) */
  TR_ENOMEM = -2,      /* device allocation failed */
  TR_EHIP = -3,        /* a HIP runtime call or launch failed */
  TR_ESINGULAR = -4,   /* S_n not positive definite / zero pivot in R_[2] */
  TR_ENONFINITE = -5   /* NaN or Inf met in M_n or in a new core */
};

/*
 * tr_als_init -- create a context for one decomposition job: the tensor and
 * initial cores of the TR format (Sec. 2) that the ALS sweeps of Alg. 1-4
 * start from, with the per-core state those updates reuse (Grams for
 * Prop. 3.1's ring product; core QRs and R-cores for Alg. 3 and Alg. 4).
 *   ctx      host out: the new context (NULL on failure).
 *   N        tensor order, 2 <= N <= 8.
 *   dims     host, I_1..I_N, each >= 1; prod(I_n) < 2^62.
 *   ranks    host, R_1..R_N, each 1..24 (R_{N+1} = R_1).
 *   X        the data tensor, prod(I_n) elements of type x_dtype, i_1 fastest.
 *            Borrowed read-only for the context's lifetime; never written or
 *            freed by the library.
 *   x_dtype  TR_F64 or TR_F32.
 *   cores    host array of N device pointers to FP64 cores in the layout above.
 *            Read here; overwritten in place at the end of each successful
 *            tr_als_sweep (stream order).  Caller-owned.
 *   variant  TR_NE, TR_QR or TR_QRNE.  For TR_QR and TR_QRNE, modes with
 *            R_n R_{n+1} > 128 factor V_n[2] by a blocked Cholesky-QR and
 *            run its large FP64 products through rocBLAS (the context holds a
 *            rocBLAS handle, created at the first such update).
 *   hip_stream  hipStream_t for all work of this context.
 * Allocates all workspace (freed by tr_als_destroy), computes ||X||_F^2 and the
 * per-core Grams (NE), core QRs (QR) or both, the Grams of the R-cores
 * (QRNE).  Synchronises the stream once.
 */
int tr_als_init(tr_als_ctx** ctx, int N, const int64_t* dims, const int64_t* ranks,
                const void* X, int x_dtype, double* const* cores, int variant,
                void* hip_stream);

/*
 * tr_als_sweep -- run nsweeps ALS sweeps; one sweep updates modes 1..N in order
 * with each new core used at once (Gauss-Seidel, Alg. 1-3).
 *   contraction_prec  TR_F64, TR_F32, TR_BF16 or TR_FP8: arithmetic of the X
 *                     contraction (MFMA with FP32 accumulation for
 *                     F32/BF16/FP8, FP64 for F64).  BF16/FP8 read a shadow copy
 *                     of X built on first use (RNE; FP8 E4M3 with one FP32
 *                     scale per tensor) and kept for the context's lifetime.
 *   refine_steps      0..4 iterative-refinement steps of the normal-equation
 *                     solve (NE and QRNE variants; ignored by TR_QR).
 * Synchronises the stream once at the end to read the device status word.
 * On TR_ESINGULAR / TR_ENONFINITE the caller's cores hold the last good mode
 * update and the context stays usable.
 */
int tr_als_sweep(tr_als_ctx* ctx, int nsweeps, int contraction_prec, int refine_steps);

/*
 * tr_als_set_solve -- how the mode update solves its least-squares problem.
 *   TR_SOLVE_FACTOR (the default): TR_NE / TR_QRNE invert S_n<2> (SPD inverse,
 *     or a blocked Cholesky for R_n R_{n+1} > 128), TR_QR substitutes with
 *     R_[2] (Alg. 3);
 *     a singular or indefinite S_n / R_[2] stops the sweep with TR_ESINGULAR.
 *   TR_SOLVE_PINV: the rank-deficient-safe solve (the remark after Alg. 3):
 *     S_n<2>^+ by a one-sided Jacobi SVD in FP64, singular values of S_n at or
 *     below rcond * max dropped (rcond = 0: R_n R_{n+1} * 2^-52), so each
 *     update is the minimum-norm least-squares solution.  TR_QR then takes
 *     Alg. 4's route through V_n[2]^T V_n[2] (a rank-deficient V_n[2] has no
 *     Cholesky-QR).  rcond in [0, 1).
 * Takes effect from the next mode update; synchronises the stream.
 */
int tr_als_set_solve(tr_als_ctx* ctx, int solve, double rcond);

/*
 * tr_als_run -- sweeps until the relative error stops improving: after each
 * sweep the error is estimated from the last mode's intermediates by the
 * identity ||X - Xhat||^2 = ||X||^2 - 2 <X, Xhat> + ||Xhat||^2 (Sec. 4, error
 * computation): <X, Xhat> = <M_N, G_N(2)> and ||Xhat||^2 = <S_N<2>, G_N(2)^T
 * G_N(2)> for TR_NE and TR_QRNE (whose M_N = Y_[N] V_N[2] and R-core Grams
 * give the same two numbers), <W_N, G_N(2) R_[2]^T> and ||G_N(2) R_[2]^T||^2
 * for TR_QR; no pass over X.  Stops after the first sweep whose estimate
 * differs from the previous sweep's by at most tol (>= 0), or after
 * max_sweeps (>= 1).
 *   sweeps_done  host out: sweeps run.
 *   rel_err      host out: the last estimate of ||X - Xhat|| / ||X||.
 * The estimate subtracts two numbers close to ||X||^2, so it loses about
 * (||X|| / ||X - Xhat||)^2 units of roundoff of M_N: use it with
 * contraction_prec = TR_F64 (in lower precisions the contraction error of M_N
 * dominates it; tr_als_fit stays exact).  Synchronises once per sweep; cores
 * written back at the end as by tr_als_sweep (also on error).
 */
int tr_als_run(tr_als_ctx* ctx, int max_sweeps, int contraction_prec, int refine_steps, double tol,
               int* sweeps_done /*host*/, double* rel_err /*host*/);

/*
 * tr_als_fit -- relative error ||X - TR(G)||_F / ||X||_F of the current cores
 * (Sec. 4 error formula), one streaming pass over X with the reconstruction
 * formed on the fly and squared differences summed in FP64.
 *   rel_err  host out.
 * Synchronises the stream.
 */
int tr_als_fit(tr_als_ctx* ctx, double* rel_err);

/* Free the context and everything it allocated.  NULL is accepted. */
int tr_als_destroy(tr_als_ctx* ctx);

/* Static text for a status code. */
const char* tr_als_strerror(int status);

/* Text of the context's last error ("" if none).  Valid until the next call on
 * the context. */
const char* tr_als_last_error(const tr_als_ctx* ctx);

/* ------------------------------------------------------------------------ *
 * Introspection of the individual hot-path steps, evaluated on the context's
 * current cores without changing them.  Outputs are device pointers the
 * caller allocates; each call synchronises the stream.
 * ------------------------------------------------------------------------ */

/* M_n = X_[n] G^{!=n}_[2] (Alg. 2 MTTSP), I_n x R_nR_{n+1}, column a + R_n*b,
 * computed by the same X-streaming kernels a sweep uses, in precision prec. */
int tr_als_mttsp(tr_als_ctx* ctx, int n /*1..N*/, int prec, double* M_out);

/* S_n<2> (R_nR_{n+1} square) from the Gram ring (Prop. 3.1). */
int tr_als_coef(tr_als_ctx* ctx, int n /*1..N*/, double* S_out);

/* Gram of core k: E[p, q] = sum_i G_k(2)[i, p] G_k(2)[i, q] (R_kR_{k+1} square). */
int tr_als_gram(tr_als_ctx* ctx, int k /*1..N*/, double* E_out);

/* One mode update (the body of a sweep for mode n), committed to the
 * context's internal cores; tr_als_store_cores copies them to the caller's
 * buffers. */
int tr_als_update_mode(tr_als_ctx* ctx, int n /*1..N*/, int prec, int refine_steps);
int tr_als_store_cores(tr_als_ctx* ctx);

/* Which X-contraction kernel a sweep uses for mode n: 1 = two-stage (a
 * tall-skinny MFMA GEMM of X against the partial-subchain table of one group
 * of memory-contiguous modes, then absorption of the remaining modes), 2 =
 * fused single pass (subchain rows formed in LDS).  Returns 1 or 2, or a
 * negative TR_E* code. */
int tr_als_mode_regime(const tr_als_ctx* ctx, int n /*1..N*/);

/* ||X||_F^2 computed at init (FP64).  host out. */
int tr_als_xnorm2(const tr_als_ctx* ctx, double* out);

/* Kernel timing of the X-streaming contraction: when enabled, every launch of
 * the X-stream kernel is bracketed by hipEvents on the context's stream; read
 * returns the summed kernel time (ms) and launch count since the last reset. */
int tr_als_profile_enable(tr_als_ctx* ctx, int enable);
int tr_als_profile_read(tr_als_ctx* ctx, double* xstream_ms /*host*/, int64_t* launches /*host*/,
                        double* bytes_per_launch /*host, algorithmic X bytes*/);

// Debugging aid.  With TR_ALS_CANARY=1 in the environment at context creation,
// every workspace buffer of a context is followed by a 4 KiB guard band filled
// with a byte pattern, and destroying the context checks the bands; returns
// the number of overrun buffers found so far in this process (each is also
// reported on stderr).  Always 0 without TR_ALS_CANARY.
int tr_als_debug_overruns(void);

// Debugging aid.  Number of sweep graphs (one per precision and refinement
// count) the context has captured and instantiated so far, or TR_EINVAL.  If
// `note` (host, `note_len` bytes) is given it receives, NUL-terminated, why the
// last capture was abandoned (empty if none was); sweeps then launch eagerly.
int tr_als_debug_graphs(const tr_als_ctx* ctx, char* note /*host, may be NULL*/, int note_len);

// Introspection of the low-precision shadows of X that the contraction reads
// (mixed precision; not a passage of the paper).  prec = TR_BF16 (BF16, round
// to nearest even from the FP32 value of each entry) or TR_FP8 (OCP E4M3 of
// float32(x) * s, one scale per tensor s = 448 / max|x|, round to nearest
// even).  transposed = 0: the shadow in X's layout, numel entries; 1: the
// transposed shadow, out[k + K r] = shadow(X[r + M k]) with K = *split_k and
// M = numel / K (TR_EINVAL when the context keeps none).  Builds the shadow if
// needed, copies it to `out` (device, numel * 2 or numel bytes, caller-owned),
// synchronises the context's stream; *scale (host) receives s (1 for BF16).
int tr_als_debug_shadow(tr_als_ctx* ctx, int prec, int transposed, void* out, float* scale /*host*/,
                        int64_t* split_k /*host, may be NULL*/);

/* ------------------------------------------------------------------------ *
 * Planted test tensors generated on the device.
 *
 * The paper's synthetic recipe (Sec. 4): TR-cores with N(0,1) entries, the
 * full tensor X_true = TR(G_1..G_N), then X = X_true + eta (||X_true|| / ||E||) E
 * with E i.i.d. N(0,1).  Every normal number comes from the counter-based
 * Philox4x32-10 generator (Salmon et al., SC'11; 10 rounds, key = seed) with the
 * Box-Muller transform: normal e of stream sid is taken from pair p = e/2 drawn
 * at counter (p mod 2^32, p / 2^32, sid, 0); words (0,1) and (2,3) give 53-bit
 * uniforms u, v = (m + 0.5) 2^-53; element 2p is sqrt(-2 ln u) cos(2 pi v),
 * element 2p+1 uses sin.  Streams: 0 the noise E (element = linear index of
 * X), 0x100 + k true core k, 0x200 + k initial core k (k = 0..N-1, element =
 * offset in the core layout above).  X_true is rounded to x_dtype, then the
 * scaled noise is added in FP64 and rounded again.
 * ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ *
 * Inner product and norm of tensors in TR format (Sec. 3.4 by-product).
 *
 * For A = TR(G_1..G_N) and B = TR(Z_1..Z_N) with the same dims, the Gram
 * tensors P_k = sum_i G_k(i)^T o Z_k(i)^T chained by general contractions hold
 * every product pair; <A, B> is the sum of the chain's entries whose two
 * left and two right indices agree (the trace of the product of the transfer
 * matrices T_k[(a,a'),(b,b')] = sum_i G_k(a,i,b) Z_k(a',i,b')).  The
 * proposition as printed takes the trace of the chain's mode-2 unfolding,
 * which is another number; this is the reading under which the identity holds.
 *   dims     host, I_1..I_N (2 <= N <= 8).
 *   ranksA / ranksB  host, ranks of each (1..24, independent of each other).
 *   coresA / coresB  host arrays of N device pointers, FP64 cores in the
 *            layout above; read only.
 *   inner / norm     host out: <A, B>, or ||A||_F = sqrt(<A, A>).
 * FP64 throughout (cross Grams on FP64 MFMA).  Allocates and frees a
 * workspace of O(sum (R_k S_k)^2) doubles; synchronises the stream.
 */
int tr_inner(int N, const int64_t* dims, const int64_t* ranksA, double* const* coresA, const int64_t* ranksB,
             double* const* coresB, double* inner /*host*/, void* hip_stream);
int tr_norm(int N, const int64_t* dims, const int64_t* ranks, double* const* cores, double* norm /*host*/,
            void* hip_stream);

/*
 * tr_gen_planted -- write the planted tensor into X (prod(I_n) elements of
 * x_dtype, TR_F32 or TR_F64).  true_cores: host array of N device pointers that
 * receive the true cores, or NULL (kept in internal workspace).  init_cores:
 * host array of N device pointers that receive N(0,1) initial cores, or NULL.
 * eta >= 0 (0: no noise).  Allocates and frees its workspace; synchronises the
 * stream.  Limits as tr_als_init.
 */
int tr_gen_planted(int N, const int64_t* dims, const int64_t* ranks, uint64_t seed, double eta, void* X,
                   int x_dtype, double* const* true_cores, double* const* init_cores, void* hip_stream);

/*
 * tr_gen_planted_noalloc -- the same generator for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): identical arguments and results, bit for
 * bit, but its workspace is a device array of TR_GEN_SCRATCH_MAX bytes inside
 * the library (one per GPU, held until the process ends), and it neither
 * allocates, frees nor synchronises: the work is only enqueued on hip_stream
 * (the caller synchronises before reading X or the cores).  Returns TR_ENOMEM,
 * without enqueuing anything, when the job's workspace exceeds
 * TR_GEN_SCRATCH_MAX (tr_gen_planted then serves it).  All calls on one GPU
 * share the array: calls that can overlap on that GPU (different streams, or
 * different host threads) race and must be serialised by the caller;
 * consecutive calls on one stream are ordered and safe.
 */
#define TR_GEN_SCRATCH_MAX ((size_t)64 << 20)
int tr_gen_planted_noalloc(int N, const int64_t* dims, const int64_t* ranks, uint64_t seed, double eta, void* X,
                           int x_dtype, double* const* true_cores, double* const* init_cores, void* hip_stream);

/* ------------------------------------------------------------------------ *
 * Serving: a request loop that runs many decomposition jobs on one GPU.
 *
 * Jobs are submitted without blocking, each with an arrival time.  A scheduler
 * thread admits arrived jobs in arrival order when a slot is free and the
 * job's whole HBM footprint (X, its BF16/FP8 shadow, cores, Grams and all
 * workspace, computed exactly before admission) fits in the server's arena;
 * a job that does not fit holds the queue for larger jobs while small jobs
 * (footprint <= arena / 64) may pass it, until it has waited 0.5 s.  Admitted
 * jobs run concurrently on their slots' streams; each keeps its cores and Gram
 * matrices resident in its arena region until it finishes.  A job runs the
 * planted-tensor generator above (or borrows the caller's X), nsweeps_mixed
 * sweeps in prec_mixed, nsweeps_fin sweeps in prec_fin, and the fit; its final
 * cores are kept on the host for tr_srv_result.  All kernels are
 * deterministic, so a job's result does not depend on what else runs.
 * With TR_SRV_BATCH, small NE jobs (order 2..4, ranks <= 8, mode sizes <= 128,
 * at most 2^18 entries, contraction FP64/FP32/BF16) skip the slots: the small
 * jobs admitted together go to an idle batch lane, where one persistent launch
 * runs each whole job (all sweeps, solve, fit) in one workgroup; two lanes
 * alternate.  A lane job's result is likewise independent of its batch.
 * All times are seconds since tr_srv_create (steady clock).
 * ------------------------------------------------------------------------ */

typedef struct tr_srv tr_srv;

enum { TR_JOB_QUEUED = 0, TR_JOB_RUNNING = 1, TR_JOB_DONE = 2, TR_JOB_FAILED = 3 };

typedef struct {
  int N;                      /* order, 2..8 */
  int64_t dims[8];            /* I_1..I_N */
  int64_t ranks[8];           /* R_1..R_N, 1..24 */
  int variant;                /* TR_NE, TR_QR or TR_QRNE */
  int prec_mixed;             /* contraction precision of the first sweeps */
  int nsweeps_mixed;
  int prec_fin;               /* contraction precision of the finishing sweeps */
  int nsweeps_fin;
  int refine;                 /* refinement steps of the NE solve, 0..4 */
  uint64_t seed;              /* generator key (X, true and initial cores) */
  double eta;                 /* relative noise of the generated X, >= 0 */
  const void* X;              /* NULL: generate; else the caller's tensor (device,
                                 borrowed read-only until the job is done) */
  int x_dtype;                /* TR_F32 or TR_F64: storage type of X */
  const double* const* init_cores; /* NULL: N(0,1) from seed; else host array of N
                                 device pointers, copied when the job starts */
  double t_arrival;           /* arrival time; earlier than the submit time = on submit */
} tr_job_desc;

typedef struct {
  int state;                  /* TR_JOB_* */
  int status;                 /* TR_OK or the failing step's code */
  double rel_err;             /* final ||X - TR(G)|| / ||X|| (NaN until done) */
  double t_arrival, t_admit, t_done;   /* t_admit/t_done < 0 until reached */
  size_t footprint;           /* HBM bytes reserved for the job */
  int slot;                   /* slot that ran it (-1 before admission) */
  int batched;                /* 1 if it ran in a batched group */
} tr_job_info;

typedef struct {
  uint64_t submitted, done, failed;
  size_t arena_bytes;         /* HBM budget */
  size_t peak_in_use;         /* largest sum of admitted footprints */
  int slots;
  int max_running;            /* most jobs admitted at once */
} tr_srv_stats;

/*
 * tr_srv_create -- start a server on the current device.
 *   hbm_budget_bytes  size of the device arena all jobs are carved from
 *                     (0: 90% of the free device memory); allocated here.
 *   max_slots         concurrent jobs, 1..64; each slot owns two streams
 *                     (default priority); one executor thread drives all
 *                     slots and is the only caller of HIP.
 *   flags             TR_SRV_BATCH: run small jobs in the batch lanes.
 * Returns TR_EINVAL, TR_ENOMEM (arena allocation) or TR_EHIP on failure.
 */
enum { TR_SRV_BATCH = 1 };
int tr_srv_create(tr_srv** srv, size_t hbm_budget_bytes, int max_slots, int flags);

/* Queue a job (host descriptor, copied).  Never blocks.  TR_EINVAL for an
 * invalid descriptor, TR_ENOMEM if its footprint exceeds the whole arena. */
int tr_srv_submit(tr_srv* srv, const tr_job_desc* desc, uint64_t* job_id /*host out*/);

/* Current state of a job (host out). */
int tr_srv_poll(tr_srv* srv, uint64_t job_id, tr_job_info* info);

/* Block until the job is done or failed; then as tr_srv_poll. */
int tr_srv_wait(tr_srv* srv, uint64_t job_id, tr_job_info* info);

/* Copy a finished job's final cores into N host arrays (layout above). */
int tr_srv_result(tr_srv* srv, uint64_t job_id, double* const* cores_host);

/* Block until every submitted job is done or failed. */
int tr_srv_drain(tr_srv* srv);

int tr_srv_stats_read(tr_srv* srv, tr_srv_stats* out /*host*/);

/* Drop queued jobs, finish running ones, free the arena and streams.  NULL is
 * accepted. */
int tr_srv_destroy(tr_srv* srv);

/* Text of the failure of a job ("" if none); valid until tr_srv_destroy. */
const char* tr_srv_job_error(tr_srv* srv, uint64_t job_id);

#ifdef __cplusplus
}
#endif
#endif /* TR_ALS_H */
