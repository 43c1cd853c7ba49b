/*
 * pasd.h - C ABI of the MI355X (gfx950) PASD solver for tensor robust PCA.
 *
 * PASD (Parallel Active Subspace Decomposition, Jiang & Ng) splits an observed
 * N-way tensor T into a low-rank part X and a sparse part E by the ADMM of
 * Algorithm 1 of the paper (Section 3.2): for every mode n the mode-n
 * unfolding of the low-rank copy Z_n is factored as U_n V_n with U_n an
 * I_n x R_n column-orthonormal "active subspace" (eq. (3)); each iteration
 * updates U_n by the orthogonal Procrustes problem (eqs. (9)-(10)), V_n by
 * singular value thresholding (eqs. (11)-(13)), E by shrinkage
 * (eqs. (14)-(15)), then the multipliers Y_n and the penalty mu, and stops when
 * every ||T - Z_n - E||_inf is below the tolerance.
 *
 * Every entry point returns an int status (enum pasd_status): 0 on success,
 * a positive warning, or a negative error.  No exception crosses the ABI.  The
 * message of the last failure on the calling thread is pasd_last_error().
 *
 * Layout: tensors are dense, row-major (C order, last mode fastest), in the
 * state dtype of the context: double for PASD_FP64, float for PASD_FP32 and
 * PASD_BF16_GEMM.  Small factors are row-major as documented per call.
 *
 * Ownership: a context owns all of its device memory from pasd_create until
 * pasd_destroy.  Buffers passed in are only read (or written) during the
 * call and may be freed afterwards; device pointers must be valid device
 * memory of the context's device.  Work is enqueued on the context's stream;
 * calls documented as synchronising wait for that stream.
 *
 * Threading: a context may be used by one thread at a time; different
 * contexts may be driven from different threads and streams concurrently.
 */
#ifndef PASD_H
#define PASD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PASD_MAX_ORDER 8   /* largest tensor order N supported */
#define PASD_MAX_RANK 64   /* largest R_n supported; I_n R_n <= 2^20 for R_n <= 16
                              and I_n R_n <= 16384 above (QR workspace) */

enum pasd_status {
  PASD_OK = 0,
  PASD_NOT_CONVERGED = 1,    /* max_iter reached before the tolerance; results valid */
  PASD_PRECISION_FLOOR = 2,  /* stopped without meeting tol: every residual fell below the
                                rounding level of the state (pasd_info.tol_effective), where
                                further iterations cannot lower it; results valid, not
                                converged in the sense of Algorithm 1 */
  PASD_ERR_INVALID_ARG = -1, /* bad pointer, dimension, rank, weight or option */
  PASD_ERR_UNSUPPORTED = -2, /* valid input outside the sizes the library handles */
  PASD_ERR_OOM = -3,         /* device allocation failed */
  PASD_ERR_HIP = -4,         /* a HIP runtime call failed */
  PASD_ERR_NUMERIC = -5,     /* a NaN or infinity appeared in the iteration */
  PASD_ERR_STATE = -6        /* call not valid in the context's current state */
};

enum pasd_precision {
  PASD_FP64 = 0,      /* FP64 state and arithmetic throughout */
  PASD_FP32 = 1,      /* FP32 state and unfolding GEMMs (FP32 MFMA); FP64 QR,
                         Gram, eigensolver, scalars */
  PASD_BF16_GEMM = 2  /* FP32 state; the unfolding GEMMs (G_n P_n^T and U_n^T G_n)
                         on the BF16 matrix cores: every FP32 operand is split
                         into three BF16 terms (round-to-nearest-even) and each
                         product is taken as six BF16 x BF16 terms with FP32
                         accumulation, which keeps FP32 accuracy; FP64 QR, Gram,
                         eigensolver, scalars; FP32 elementwise pass */
};

/* Solver configuration.  pasd_config_init() fills every field with its
 * default; callers then set order, dims and ranks at least. */
typedef struct {
  int order;                        /* N, 2 <= N <= PASD_MAX_ORDER */
  int64_t dims[PASD_MAX_ORDER];     /* I_1..I_N, each >= 1 */
  int64_t ranks[PASD_MAX_ORDER];    /* R_n, 1 <= R_n <= min(I_n, J_n, PASD_MAX_RANK),
                                       J_n = prod_{m != n} I_m (eq. (3): r_n <= R_n) */
  double lambda[PASD_MAX_ORDER];    /* nuclear-norm weights lambda_n of eq. (3); a value
                                       <= 0 selects sqrt(max(I_n, J_n)) / N (Section 5.1) */
  double alpha[PASD_MAX_ORDER];     /* output weights alpha_n of Algorithm 1; a value
                                       <= 0 selects alpha_n = lambda_n */
  double mu0;                       /* initial penalty, default 1e-4 (Algorithm 1) */
  double mu_max;                    /* penalty cap, default 1e10 (Algorithm 1) */
  double rho;                       /* penalty growth, default 1.1 (Algorithm 1) */
  double tol;                       /* epsilon of the stopping test, default 1e-5; 0 disables
                                       the test (the solve runs to max_iter) */
  int max_iter;                     /* iteration cap, default 1000 (Section 5.1) */
  int precision;                    /* enum pasd_precision, default PASD_FP64 */
  int device;                       /* HIP device ordinal; -1 = current device */
  void *stream;                     /* hipStream_t for all work; NULL = null stream */
  int flags;                        /* bitwise OR of enum pasd_flags, default 0 */
} pasd_config;

enum pasd_flags {
  PASD_FLAG_NO_GRAPH = 1,     /* launch every kernel directly instead of replaying a captured
                                 HIP graph of 16 iterations (same results, bitwise) */
  PASD_FLAG_TIEBREAK_KEEP = 2, /* Procrustes tie-break of eq. (10) when V_n^k is rank deficient:
                                 span U_n^{k+1} = range(G_n^k (V_n^k)^T) plus, on the directions
                                 where V_n^k vanishes, the previous U_n^k (the maximiser of
                                 eq. (10) nearest U_n^k).  Default (flag clear): span U_n^{k+1}
                                 = range(G_n^k (P_n^k)^T) with the pre-threshold P_n^k.  Both
                                 agree while every V_n^k has full rank; at k = 0 both keep U^0 */
  PASD_FLAG_NO_FLOOR_STOP = 4  /* do not stop at the precision floor (done = 4): iterate until
                                  Algorithm 1's test holds or max_iter */
};

/* Progress and status of a context. */
typedef struct {
  int iterations;                   /* completed ADMM iterations k */
  int converged;                    /* 1 once max_n residual[n] < tol (Algorithm 1, line 8) */
  int done;                         /* 0 running, 1 converged, 2 max_iter, 3 numeric error,
                                       4 stopped at the precision floor (see tol_effective) */
  double mu;                        /* current penalty mu^k */
  double residual[PASD_MAX_ORDER];  /* ||T - Z_n - E||_inf of the last iteration */
  int rank[PASD_MAX_ORDER];         /* #{singular values of U_n^T G_n above lambda_n/mu}
                                       in the last SVT, per mode */
  size_t bytes_resident;            /* device memory held by the context */
  int eig_sweeps[PASD_MAX_ORDER];   /* Jacobi sweeps of the last Gram eigensolve, per mode */
  double tol_effective;             /* precision floor of the last stopping test,
                                       max(tol, c u max|T - E|) with u the unit roundoff of the
                                       state: the N low-rank copies, each a sum of R_n rounded
                                       rank terms, cannot agree beyond a few units of the last
                                       place (measured floors 8-12 u max|T - E| in FP32), so
                                       c u = 16 * 2^-24 for an FP32 state (also with split-BF16
                                       GEMM operands) and 8 * 2^-53 in FP64.  A solve whose
                                       residuals all fall below it but not below tol stops with
                                       done = 4 and converged = 0 (PASD_PRECISION_FLOOR) unless
                                       PASD_FLAG_NO_FLOOR_STOP is set */
  int merged_modes;                 /* modes 0 .. merged_modes-1 whose G_n P_n^T (eq. (10)) the
                                       fused pass of the previous iteration accumulates instead
                                       of a separate unfolding GEMM: 0, 2 (order-4 tensors whose
                                       last two dimensions hold at least 1024 vectors; FP32
                                       states up to rank 10) or 4 (also the last two modes: FP64
                                       state, ranks up to 6, rows of at most 64 vectors) */
  int fused_blocks;                 /* workgroups of one launch of the fused pass */
  int gemm_p_pair;                  /* 1: P_n = U_n^T G_n (eq. (13)) of the last two modes
                                       runs as one pass over their 64 x 64 slabs, reading
                                       D = T - E once for both (order >= 3, I_{N-2} = I_{N-1}
                                       = 64, every R_n <= 16, not with split-BF16 operands) */
} pasd_info;

typedef struct pasd_ctx pasd_ctx;

/* Quantities that pasd_export / pasd_import move (checkpoint, inspection). */
enum pasd_quantity {
  PASD_Q_E = 0,      /* sparse part E (numel, state dtype) */
  PASD_Q_Y = 1,      /* multiplier Y_n (numel, state dtype), index = n */
  PASD_Q_Z = 2,      /* low-rank copy Z_n = fold_n(U_n V_n) (numel, state dtype), export only */
  PASD_Q_X = 3,      /* output X = sum alpha_n Z_n / sum alpha_n (numel, state dtype), export only */
  PASD_Q_U = 4,      /* active subspace U_n, I_n x R_n row-major, double */
  PASD_Q_P = 5,      /* P_n = U_n^T G_n, R_n x J_n row-major, state dtype; V_n = SVT(P_n) */
  PASD_Q_UF = 6,     /* U_n W_n with W_n the R_n x R_n SVT factor (V_n = W_n P_n),
                        I_n x R_n row-major, double, export only */
  PASD_Q_SCALARS = 7, /* double[2] = {k, mu} */
  PASD_Q_D = 8,       /* D = T - E as the solver stores it (numel, state dtype); a
                         checkpoint of D (not E) restores the iterate bitwise */
  PASD_Q_WEV = 9,     /* eigenvectors of the last Gram P_n P_n^T, the starting basis
                         of the next eigensolve: R_n x R_n row-major, double */
  PASD_Q_FAC = 10     /* SVT weights f_i = (s_i - tau)_+ / s_i of the last eigensolve, in the
                         order of the columns of PASD_Q_WEV: R_n doubles (the keep tie-break
                         of PASD_FLAG_TIEBREAK_KEEP reads them at the next iteration) */
};

/* Fill cfg with defaults (order 0, no dims).  Host only. */
int pasd_config_init(pasd_config *cfg);

/* Check cfg without touching any device (host only).  Returns PASD_OK,
 * PASD_ERR_INVALID_ARG or PASD_ERR_UNSUPPORTED; never a HIP error. */
int pasd_validate(const pasd_config *cfg);

/* Device bytes a context for cfg would allocate (host only); used for
 * admission by footprint. */
int pasd_footprint(const pasd_config *cfg, size_t *bytes);

/* Create a context: validates cfg on the host, allocates the solver state on
 * the device and copies T in (row-major, state dtype; T_on_device says
 * whether T is a device or host pointer).  The state is set to the
 * initialisation of Algorithm 1.  On failure *out is NULL. */
int pasd_create(const pasd_config *cfg, const void *T, int T_on_device, pasd_ctx **out);

/* Return the context to the initialisation of Algorithm 1 (k = 0) without
 * reallocating; T is kept.  Asynchronous. */
int pasd_reset(pasd_ctx *ctx);

/* Enqueue n_iters ADMM iterations (Algorithm 1, lines 2-8) on the context's
 * stream.  Asynchronous: iterations after convergence, after max_iter or
 * after a numeric error are skipped on the device. */
int pasd_step(pasd_ctx *ctx, int n_iters);

/* Iterate until converged, max_iter or the precision floor (synchronising),
 * then fill info if non-NULL.  Returns PASD_OK if Algorithm 1's test
 * max_n ||T - Z_n - E||_inf < tol held, PASD_NOT_CONVERGED at max_iter,
 * PASD_PRECISION_FLOOR when the residuals stalled below the state's rounding
 * level but above tol, PASD_ERR_NUMERIC on NaN/Inf. */
int pasd_solve(pasd_ctx *ctx, pasd_info *info);

/* Synchronise and report progress. */
int pasd_query(pasd_ctx *ctx, pasd_info *info);

/* Output of Algorithm 1: X = sum_n alpha_n Z_n / sum_n alpha_n and E, into
 * caller buffers of numel elements in the state dtype (either may be NULL).
 * Synchronising. */
int pasd_get_result(pasd_ctx *ctx, void *X, void *E, int on_device);

/* Copy one quantity out (see enum pasd_quantity; index = mode n where it
 * applies).  Synchronising. */
int pasd_export(pasd_ctx *ctx, int quantity, int index, void *dst, int dst_on_device);

/* Overwrite one quantity (E or D, Y_n, U_n, P_n, the eigenbasis or the
 * scalars) for checkpoint restore.  A restore of D, every Y_n, U_n, P_n, the
 * eigenbases and the scalars reproduces the saved iterate bitwise (E is
 * converted to D = T - E, which is exact only up to rounding; without the
 * eigenbases the continuation agrees to rounding).  Synchronising. */
int pasd_import(pasd_ctx *ctx, int quantity, int index, const void *src, int src_on_device);

/* Step several contexts together (serving): n_iters iterations of each,
 * enqueued so that independent contexts overlap on the device.  Contexts
 * must be distinct and on the same device.  Asynchronous. */
int pasd_step_batch(pasd_ctx *const *ctxs, int count, int n_iters);

/* A captured batched step (serving): pasd_batch_create records n_iters
 * iterations of every context of the list, grouped exactly as
 * pasd_step_batch groups them, into one HIP graph (captured on a private
 * stream; nothing runs during the call); pasd_batch_step replays it on the
 * contexts' common stream (asynchronous), advancing each context that is
 * still running by n_iters iterations with the same results, bitwise, as
 * pasd_step_batch.  The graph holds the contexts' device state: every context
 * must stay alive, unchanged in membership, until pasd_batch_destroy, and a
 * context that has finished (converged, max_iter, floor) is skipped on the
 * device.  A serving loop re-creates the batch when its resident set changes.
 * Errors: PASD_ERR_INVALID_ARG for the lists pasd_step_batch rejects or an
 * empty list; PASD_ERR_HIP if capture or instantiation fails (*out NULL). */
typedef struct pasd_batch pasd_batch;
int pasd_batch_create(pasd_ctx *const *ctxs, int count, int n_iters, pasd_batch **out);
int pasd_batch_step(pasd_batch *batch);
void pasd_batch_destroy(pasd_batch *batch);   /* NULL-safe */

/* Kernels of one iteration, in launch order (indices of pasd_profile). */
enum pasd_kernel {
  PASD_K_GEMM_M = 0,  /* M_n = G_n P_n^T split-K partials (eq. (10) operand) */
  PASD_K_REDUCE_M,    /* fixed-order reduction of the partials */
  PASD_K_QR,          /* U_n = orthonormal basis of range(M_n) (CholeskyQR2 or Householder;
                         with PASD_FLAG_TIEBREAK_KEEP the tie-break transform of M_n first) */
  PASD_K_GEMM_P,      /* P_n = U_n^T G_n (eq. (13) operand) */
  PASD_K_GRAM,        /* S_n = P_n P_n^T partials */
  PASD_K_EIG,         /* Jacobi eigensolver of S_n, SVT factor */
  PASD_K_FUSED,       /* Z_n, E (eq. (15)), Y_n, residuals in one pass */
  PASD_K_CONTROL,     /* mu, k, stopping test */
  PASD_NUM_KERNELS
};

/* Run n_iters iterations like pasd_step with a HIP event recorded between
 * consecutive kernel launches on the context's stream; synchronises and adds
 * the elapsed milliseconds of each launch to ms[kind] and the launch count to
 * launches[kind] (arrays of PASD_NUM_KERNELS; launches may be NULL; both are
 * zeroed first).  Iterations skipped after convergence still count. */
int pasd_profile(pasd_ctx *ctx, int n_iters, double *ms, int *launches);

/* pasd_query for several contexts with a single synchronisation per stream
 * (serving loops poll every resident solve after each batched step). */
int pasd_query_batch(pasd_ctx *const *ctxs, int count, pasd_info *infos);

/* One whole solve that allocates nothing, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc).
 * Equivalent to pasd_create + pasd_solve + pasd_get_result + pasd_destroy on
 * a context with PASD_FLAG_NO_GRAPH (the same kernels in the same order,
 * launched directly on cfg->stream, so the same results), except that T is
 * read in place and the solver state lives in a static device array of
 * pasd_static_scratch_bytes() bytes (32 MiB) that the library holds on every
 * GPU it runs on until the process ends.
 *   T    device pointer, numel elements of the state dtype, row-major; only
 *        read, and must stay valid until the call returns.
 *   X, E device pointers receiving the output of Algorithm 1 (numel elements
 *        of the state dtype each); either may be NULL.
 *   info filled as by pasd_solve when non-NULL.
 * Returns pasd_solve's status (results are written for PASD_OK,
 * PASD_NOT_CONVERGED and PASD_PRECISION_FLOOR), PASD_ERR_INVALID_ARG, or
 * PASD_ERR_UNSUPPORTED when the state does not fit the static array (it takes
 * pasd_footprint(cfg) minus two tensors of numel elements).  Calls no
 * hipMalloc, hipFree, graph instantiation or other allocating routine; the
 * state is cleared at the start of every call.  Synchronising.  All calls on
 * one GPU share its array: calls that overlap on the same GPU (from several
 * threads or streams) race and must be serialised by the caller. */
int pasd_solve_static(const pasd_config *cfg, const void *T, void *X, void *E, pasd_info *info);

/* Size in bytes of the static device array behind pasd_solve_static. */
size_t pasd_static_scratch_bytes(void);

/* Release everything the context holds.  NULL-safe. */
void pasd_destroy(pasd_ctx *ctx);

/* Message of the last failure on the calling thread ("" if none). */
const char *pasd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PASD_H */
