/*
 * svt.h -- C-ABI of the MI355X (gfx950) implementation of fast singular value
 * thresholding with recycling rank-revealing randomized SVD (R4SVD).
 *
 * Paper: Y. Li, W. Yu, "A Fast Implementation of Singular Value Thresholding
 * Algorithm using Recycling Rank Revealing Randomized Singular Value
 * Decomposition" (arXiv 1704.05528).
 *
 * Problem (Sec. 1, Eq. 1-3): complete an m x n matrix A from its entries on an
 * observed set Lambda.  SVT iterates (Eq. 4)
 *     X^(i)   = D_tau(Y^(i))                       (Eq. 5, soft-thresholded SVD)
 *     Y^(i+1) = Y^(i) + delta * P_Lambda(A - X^(i))
 * where Y lives on Lambda only and X is never formed densely.  D_tau(Y) is
 * evaluated by R4SVD (Sec. 2.4, Alg. 3): the left singular vectors of the
 * previous iteration are recycled as the starting basis Q, and Gaussian blocks
 * of Delta-t columns orthogonal to Q are appended until the error percentage
 * (||Y||_F^2 - ||Q^T Y||_F^2) / ||Y||_F^2 (Eq. 8, 10, 11) falls to
 * eps_threshold.  The first iteration starts from a t-column block (R3SVD,
 * Alg. 2).  eps_threshold is multiplied by beta whenever the residual fails to
 * decrease (Sec. 2.5, Eq. 13-14, Alg. 4).
 *
 * Conventions
 *  - All pointers in these calls are HOST pointers unless a parameter or flag
 *    says otherwise (svt_init's ptr_is_device, svt_factors's out_is_device,
 *    svt_sample's ptr_is_device, SVT_GRAD_DEVICE_POINTERS, svt_mae_device).
 *    Device pointers must be memory of the handle's device; work on them is
 *    ordered on the handle's stream.  Inputs are copied; the library keeps no
 *    caller pointer.
 *  - Index arrays are 0-based int32.  Lambda is given as COO (rows[p], cols[p]),
 *    p = 0..nnz-1, in any order, without duplicates.  Vectors "on Lambda"
 *    (values, y, x, residuals) are in that caller order.
 *  - Dense matrices crossing the ABI are row-major float64.
 *  - Every call returns an svt_status.  On error the outputs are unspecified,
 *    svt_last_error() describes the failure, and the handle stays usable
 *    unless the status is SVT_E_HIP.
 *  - Non-convergence is not an error; it is reported in svt_step_stats.flags.
 *  - A handle is bound to the device that was current at svt_init and to the
 *    stream given there.  Calls on one handle must not overlap.
 */
#ifndef SVT_H
#define SVT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct svt_handle svt_handle;

typedef enum {
  SVT_OK = 0,
  SVT_E_INVALID_ARG = -1, /* bad size, index out of range, duplicate entry, bad parameter */
  SVT_E_OOM = -2,         /* device or host allocation failed */
  SVT_E_HIP = -3,         /* a HIP runtime call failed; the handle must be destroyed */
  SVT_E_NUMERIC = -4,     /* NaN/Inf in a reduction or in the projected Gram's eigenvalues (an iterate that
                             has left the storage type's range, e.g. under a step size above the stable
                             bound), or a non-positive ||Y||_F */
  SVT_E_STATE = -5,       /* call not valid in the handle's current state */
  SVT_E_LIMIT = -6        /* more singular values above tau than the tracked maximum (kmax), or a basis
                             wider than the full eigen-solver's largest order (4096) */
} svt_status;

/* Precision forms. */
enum {
  SVT_FP64 = 0,  /* every stored value and every accumulation in float64 */
  SVT_MIXED = 1, /* float32 storage of y, a, Q, W, sampled blocks and factors, float32 accumulation in
                    the sparse products and the sampled update; float64 Gram matrices, Cholesky,
                    eigen-solver and every norm and reduction */
  SVT_BF16 = 2   /* SVT_MIXED with the basis Q stored in bfloat16 (each sampled block orthonormalised
                    in float32, then rounded to nearest even).  The rounded basis is not orthonormal,
                    so the projection of Alg. 3 is taken on the exact orthogonal projector onto its
                    span: with Q^T Q = L L^T (float64 Cholesky, bordered as blocks are appended),
                    ||B||_F^2 of Eq. 10-11 is trace(L^-1 W^T W L^-T) and svd(B) is taken through the
                    eigenpairs of L^-1 W^T W L^-T.  The whole stored basis is recycled (no truncated
                    recycling); svt_grad is not available */
};

/* Operator variants (svt_params.mode). */
enum {
  SVT_MODE_R4SVD = 0, /* Alg. 3: recycle the previous left singular vectors (Sec. 2.4), default */
  SVT_MODE_R3SVD = 1, /* Alg. 2 from a fresh t-block in every SVT iteration (no recycling, Sec. 2.2) */
  SVT_MODE_RSVD = 2   /* Alg. 1: fixed-rank randomized SVD with rank + oversample Gaussian samples,
                         no growth, the `rank` leading singular triplets thresholded (Sec. 2.1) */
};

/* Bits of svt_step_stats.flags. */
enum {
  SVT_F_CONVERGED = 1, /* relative residual fell below tol; Y was not updated */
  SVT_F_MAXIT = 2,     /* svt_iterate reached maxit */
  SVT_F_RMAX_HIT = 4,  /* growth stopped because the basis reached r_max */
  SVT_F_EXHAUSTED = 8, /* a growth block had no direction outside span(Q) */
  SVT_F_ANNEALED = 16, /* eps_threshold was multiplied by beta in this iteration */
  SVT_F_EIG_INEXACT = 32, /* the eigen-solver stopped at its cap (products of the subspace solver, or
                             sweeps of the full decomposition) */
  SVT_F_DIVERGING = 64     /* the relative residual has stayed above 10 times its smallest value so far for
                             5 iterations in a row (annealing, the paper's only response to a residual that
                             stops decreasing, cannot correct a step size above the stable bound) */
};

/* Inputs of Alg. 4 plus the values the paper leaves open.  Fill with
 * svt_default_params() and override.  "<= 0 => default" fields take the
 * paper's experimental settings of Sec. 3 where it gives them. */
typedef struct {
  double tau;      /* threshold parameter tau (> 0) */
  double delta;    /* step size delta (> 0) */
  double tol;      /* stop when ||P_Lambda(A - X)||_F / ||P_Lambda A||_F < tol */
  double beta;     /* annealing factor, 0 < beta < 1 (Sec. 3: 0.95) */
  double eta;      /* residual counts as decreasing only if rel < eps_min * (1 - eta); default 0 */
  double eps_thr0; /* initial eps_threshold; < 0 => (1 + eps_1) / 2 with eps_1 from the first t-block */
  int32_t maxit;   /* iteration cap for svt_iterate (default 500) */
  int32_t t0;      /* first block width t; <= 0 => floor(0.05 min(m, n)), at least 1 */
  int32_t dt;      /* growth block width Delta-t; <= 0 => 10 */
  int32_t npow;    /* power iterations per sampled block, X <- Y (Y^T X) after re-orthonormalisation */
  int32_t r_max;   /* basis width cap; <= 0 => m */
  int32_t k0;      /* kicking count; < 0 => ceil(tau / (delta ||P_Lambda A||_2)) */
  uint64_t seed;   /* key of the Philox4x64-10 Omega stream */
  int32_t precision; /* SVT_FP64, SVT_MIXED or SVT_BF16 */
  int32_t kmax;    /* most singular values above tau tracked (the factor buffers hold this many
                      columns); <= 0 => r_max, i.e. every singular value the basis can hold.  Counts
                      that need a wider block than the subspace solver's 96 columns are found by a full
                      eigen-decomposition of the projected Gram (Jacobi over many workgroups) */
  int32_t mode;    /* SVT_MODE_R4SVD (default), SVT_MODE_R3SVD or SVT_MODE_RSVD */
  int32_t recycle_extra; /* R4SVD: < 0 recycles all r columns (default); e >= 0 recycles only the
                            k + e leading left singular vectors of B */
  int32_t rank;    /* SVT_MODE_RSVD: the fixed rank (> 0) */
  int32_t oversample; /* SVT_MODE_RSVD: oversampling p >= 0 (default 10) */
  double mae_tol;  /* > 0: also stop when the sample MAE (1/|Lambda|) sum |A - X| on Lambda falls
                      below mae_tol (the stop rule of Sec. 3); <= 0: unused */
  double wait_timeout_s; /* longest host wait for the device at one decision point; <= 0 => 600 s.  A
                            wait that runs out returns SVT_E_HIP and marks the handle lost:
                            svt_destroy then neither waits for its stream nor frees its device
                            memory (a kernel may still be using it) */
} svt_params;

/* Per-iteration report. */
typedef struct {
  int32_t iter;      /* SVT iteration number i (1-based) */
  int32_t r;         /* basis width after R4SVD */
  int32_t k;         /* number of singular values of B above tau */
  int32_t blocks;    /* growth blocks appended in this iteration */
  int32_t annealed;  /* 1 if eps_threshold was multiplied by beta */
  int32_t stopped;   /* 1 if rel_res < tol (Y not updated) */
  int32_t flags;     /* SVT_F_* bits */
  int32_t eig_iters; /* products and tests of the subspace eigen-solver, or the sweeps of the full
                        Jacobi decomposition of the projected Gram */
  double eps;        /* error percentage when R4SVD returned */
  double eps_thr;    /* eps_threshold R4SVD ran with */
  double rel_res;    /* ||P_Lambda(A - X)||_F / ||P_Lambda A||_F */
  double normY;      /* ||Y||_F^2 */
  double normB;      /* ||Q^T Y||_F^2 */
  double sigma1;     /* largest singular value of B */
  double sigmak;     /* smallest singular value above tau (0 if k = 0) */
  double grow_margin;   /* min over growth tests of |eps - eps_thr| / eps_thr */
  double anneal_margin; /* (rel - eps_min (1 - eta)) / eps_min before the update */
  double mae;           /* sample MAE (1/|Lambda|) sum |A - X| on Lambda (Sec. 3) */
} svt_step_stats;

/* Fill *p with defaults (tau and delta are set to 0 and must be given). */
void svt_default_params(svt_params* p);

/* Element types of the observed values given to svt_init. */
enum {
  SVT_DTYPE_F64 = 0, /* double */
  SVT_DTYPE_F32 = 1  /* float; widened to double on input */
};

/* Create a handle for the problem (Alg. 4 inputs).  Copies the COO triplets
 * (rows, cols: int32; vals: nnz values of type vals_dtype) to the device, builds the column-major (CSC) and row-major (CSR) orders,
 * computes ||P_Lambda A||_F and, when p->k0 < 0, ||P_Lambda A||_2 by power
 * iteration, and sets Y^(0) = k0 * delta * P_Lambda(A) (kicking, Alg. 4
 * initialisation).  stream: a hipStream_t, or NULL for the default stream; every
 * later call on the handle works on it, so it must stay valid until svt_destroy.
 * ptr_is_device = 1: rows, cols and vals are device pointers; they are read
 * once, on the given stream, before the call returns (the orders of Lambda and
 * the checks are built on the host either way).
 * Errors: SVT_E_INVALID_ARG for m, n, nnz <= 0, indices out of range,
 * duplicate (row, col), tau <= 0, delta <= 0, beta outside (0, 1), eta outside
 * [0, 1), npow < 0, non-finite values, an unknown vals_dtype, ptr_is_device
 * other than 0 or 1; SVT_E_HIP when the device inputs cannot be read. */
svt_status svt_init(svt_handle** out, int64_t m, int64_t n, int64_t nnz, const int32_t* rows,
                    const int32_t* cols, const void* vals, int32_t vals_dtype, int32_t ptr_is_device,
                    const svt_params* p, void* stream);

/* One R4SVD (Alg. 3; Alg. 2 when no basis exists yet) on the current iterate
 * Y, followed by the thresholded factors of D_tau(Y) (Eq. 5).  The iteration
 * state (Y, basis, thresholds, counters) is left unchanged; the factors can be
 * read with svt_factors.  Uses the Omega blocks of the next iteration. */
svt_status r4svd_step(svt_handle* h, svt_step_stats* st);

/* Up to max_steps iterations of Alg. 4, stopping early at convergence or at
 * maxit.  *last receives the report of the last iteration run (may be NULL).
 * Returns SVT_E_STATE if the run had already converged, SVT_E_NUMERIC when the
 * iterate stops being finite (a diverging step size), SVT_E_LIMIT when more than
 * kmax singular values rise above tau.  In R4SVD mode, unless the run stopped,
 * the call returns with the next step's first kernels (the projection of the
 * new iterate on the recycled basis) queued on the handle's stream; later calls
 * on the handle are ordered after them. */
svt_status svt_iterate(svt_handle* h, int32_t max_steps, svt_step_stats* last);

/* Reports of the iterations run by svt_iterate on this handle, oldest first (iteration i of the
 * run is record i - 1; replacing the state with svt_set_state does not clear them).  *total
 * (may be NULL) receives the number of records; out[0 .. count) receives records first ..
 * first + count - 1 that exist.  Host memory only; no device work.
 * Errors: SVT_E_INVALID_ARG (first < 0, count < 0, out == NULL with count > 0). */
svt_status svt_history(const svt_handle* h, int64_t first, int64_t count, svt_step_stats* out, int64_t* total);

/* Thresholded factors of the last X = U diag(s) V^T (s = sigma - tau > 0):
 * k (host) receives their count; U (m x kcap), V (n x kcap) row-major and s
 * (kcap) receive min(k, kcap) columns; columns kcap beyond that are left as
 * they were.  Any output pointer may be NULL.  out_is_device = 1: s, U and V
 * are device pointers, written on the handle's stream (the call returns once
 * s has been copied; U and V are ordered before later work on that stream). */
svt_status svt_factors(svt_handle* h, int32_t kcap, int32_t* k, double* s, double* U, double* V,
                       int32_t out_is_device);

/* X of the last iteration sampled on nq arbitrary entries (qi[l], qj[l]).
 * ptr_is_device = 0: host arrays; an index outside m x n is SVT_E_INVALID_ARG
 * and nothing is written.  ptr_is_device = 1: device arrays; nothing is
 * allocated, the call only enqueues one kernel on the handle's stream and
 * returns, and an index outside m x n gives NaN at its place (the other
 * entries are computed). */
svt_status svt_sample(svt_handle* h, int64_t nq, const int32_t* qi, const int32_t* qj, double* x_out,
                      int32_t ptr_is_device);

/* Mean absolute error of the last X against reference values ref on nq entries (qi[l], qj[l]):
 * *mae = (1/nq) sum_l |ref[l] - X(qi[l], qj[l])|, the MAE of Eq. 15 restricted to the given entries
 * (all m n entries for the overall error, a held-out set for a test error).  nq >= 1. */
svt_status svt_mae(svt_handle* h, int64_t nq, const int32_t* qi, const int32_t* qj, const double* ref, double* mae);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): svt_mae with DEVICE pointers and no allocation, host
 * copy or host synchronisation.  qi, qj (int32) and ref (float64) hold nq entries in device memory;
 * mae points to one float64 in device memory that receives (1/nq) sum_l |ref[l] - X(qi[l], qj[l])|,
 * the same value svt_mae returns.  The work is enqueued on the handle's stream and the call returns
 * without waiting.  The reduction keeps its partial sums in a fixed library scratch array of 1032
 * doubles in each GPU's memory (held until the process ends); every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (other handles, other streams) race.  An index out
 * of range gives a NaN result (the kernel checks every index before reading).
 * Errors: SVT_E_INVALID_ARG (nq outside [1, 2^31 - 1], a NULL pointer), SVT_E_STATE (no factors). */
svt_status svt_mae_device(svt_handle* h, int64_t nq, const int32_t* qi, const int32_t* qj, const double* ref,
                          double* mae);

/* Current state: y (nnz, caller order), basis Q (m x r row-major; pass
 * qcap >= r columns, or NULL), r, eps_threshold (NaN before the first
 * iteration), eps_min, iterations completed. */
svt_status svt_get_state(svt_handle* h, double* y, double* Q, int32_t qcap, int32_t* r, double* eps_thr,
                         double* eps_min, int32_t* iter);

/* Replace the state (for step-by-step comparisons and restarts).  Q (m x r
 * row-major, orthonormal columns) may be NULL with r = 0.  eps_thr NaN means
 * "not yet fixed".  iter is the number of iterations already completed; the
 * next iteration draws the Omega blocks of iteration iter + 1. */
svt_status svt_set_state(svt_handle* h, const double* y, const double* Q, int32_t r, double eps_thr,
                         double eps_min, int32_t iter);

/* Checkpoint for restarts: everything the next iterations read, in one host blob (Y on Lambda,
 * the basis, the thresholds and counters, the eigen-solvers' warm-start vectors, the factors of the
 * last X, and the decision log: the step reports, the basis widths and sampled blocks of every
 * iteration, and the replay queue).  A handle restored from it continues bit for bit as the
 * checkpointed one would, and svt_grad works across the restore.  buf = NULL: *size receives the
 * bytes needed; otherwise cap must be at least that.  The blob's layout is this library's own
 * (host byte order), not a stable file format.
 * Errors: SVT_E_INVALID_ARG (size NULL, cap too small). */
svt_status svt_checkpoint(svt_handle* h, void* buf, int64_t cap, int64_t* size);

/* Load a checkpoint into a handle created by svt_init for the same problem (m, n, observed set and
 * values), precision form, r_max and kmax.  Errors: SVT_E_INVALID_ARG (not a checkpoint, another
 * problem or form, malformed; the handle is then unchanged). */
svt_status svt_restore(svt_handle* h, const void* buf, int64_t size);

/* Force the two discrete decisions of the next len iterations: blocks[l]
 * growth blocks and annealed[l] (0/1).  len = 0 clears the replay. */
svt_status svt_set_replay(svt_handle* h, const int32_t* blocks, const int32_t* annealed, int32_t len);

/* Flags of svt_grad. */
enum {
  SVT_GRAD_FROZEN_BASIS = 1,   /* hold every basis Q_i of the forward run fixed (see svt_grad) */
  SVT_GRAD_DEVICE_POINTERS = 2 /* hi, hj, gx_h and da are device pointers (dtau, ddelta stay host) */
};

/* Derivative of a held-out loss through the first T unrolled iterations of
 * Alg. 4 (Eq. 4 with the kicking start).  The kicking count and every growth
 * and annealing decision of the forward run are held fixed (they are discrete).
 *
 * Default (flags = 0): the exact derivative of the iteration as R4SVD computes
 * it.  Iteration i maps Y_i to X_i = Q_i D_tau(Q_i^T Y_i) (Eq. 5) with the
 * basis Q_i itself a function of the iterates: the recycled basis of iteration
 * i - 1 (Alg. 3) followed by the sampled blocks orthonormalised against it
 * (Alg. 2-3), each a function of Y_i Omega.  The reverse sweep carries the
 * cotangent of the recycled basis from iteration to iteration.  It needs the
 * R4SVD mode with every column recycled (recycle_extra < 0), npow = 0 and no
 * column dropped by the orthonormalisation since svt_init.
 *
 * SVT_GRAD_FROZEN_BASIS: every basis Q_i is held fixed as well, so iteration i
 * is the map Y_i -> Q_i D_tau(Q_i^T Y_i) of a constant Q_i.  This leaves out the
 * basis's dependence on the iterates; it equals the exact derivative only when
 * no block is sampled from an iterate that depends on the inputs.
 *
 * The handle must have run at least T iterations since svt_init (svt_iterate,
 * no svt_set_state since), in the FP64 form.  Every eigenpair of each projected
 * Gram enters the derivative: bases up to 96 columns are diagonalised in one
 * workgroup, wider ones (up to 4096) by the many-workgroup Jacobi.  The Y_i are
 * recomputed from Y_1 = k0 delta P(A), checkpointed every ckpt iterations
 * (ckpt <= 0: about sqrt(T)); device memory of (T / ckpt + ckpt) nnz doubles
 * plus blocks of m x 3w and n x 3w doubles (w = the widest basis plus 2, rounded
 * up to 8) and a few w x w matrices is allocated for the call and released
 * before it returns.
 * Input: gx_h[l] = dL/dX_T(hi[l], hj[l]) on the held-out set H (nh entries,
 * repeats add up; nh = 0 gives zero gradients).
 * Outputs: *dtau, *ddelta, and da (nnz, caller order) = dL/dA on Lambda.
 * With SVT_GRAD_DEVICE_POINTERS the held-out arrays are read from the device
 * and da is written there; the call returns when da is complete.
 * The iteration state of the handle is left unchanged.
 * Errors: SVT_E_INVALID_ARG (T <= 0, NULL outputs, H index out of range,
 * unknown flags), SVT_E_STATE (fewer than T recorded iterations, state
 * replaced, mixed form; for the exact derivative also another mode, truncated
 * recycling, power iterations or a dropped column), SVT_E_LIMIT (a basis wider
 * than 4096 columns), SVT_E_NUMERIC (an eigen-decomposition that did not
 * converge). */
svt_status svt_grad(svt_handle* h, int32_t T, int32_t ckpt, int64_t nh, const int32_t* hi, const int32_t* hj,
                    const double* gx_h, int32_t flags, double* dtau, double* ddelta, double* da);

/* Instrumentation.  Phases of one iteration whose device time can be measured with hipEvents
 * recorded on the handle's stream around the launches of that phase. */
enum {
  SVT_PH_SPMM_T = 0,  /* W = Y^T Q on the recycled basis (one kernel: sparse, or dense on the copy of Y) */
  SVT_PH_GROW = 1,    /* growth blocks: Omega, Y Omega, projections, CholeskyQR2, Y^T Q' */
  SVT_PH_GRAM = 2,    /* G = W^T W */
  SVT_PH_EIG = 3,     /* eigenpairs of G above tau^2 (Jacobi / block subspace iteration) */
  SVT_PH_FACTORS = 4, /* Ut = Q C, Vt = W D */
  SVT_PH_SDDMM = 5,   /* fused sampled product, residual and dual update (one kernel) */
  SVT_PH_REDUCE = 6,  /* norms and their deterministic final sums */
  SVT_PH_DENSIFY = 7, /* scatter of y into the dense transposed copy of Y (dense path only) */
  SVT_PH_COUNT = 8
};

/* enable = 1 resets the counters and starts recording every phase; enable = 0 stops.  Recording
 * adds two hipEventRecord calls per measured phase instance, each a marker the GPU processes
 * between kernels (a few microseconds): record only the phases of interest with
 * svt_profile_phases when the iteration rate is measured at the same time. */
svt_status svt_profile(svt_handle* h, int32_t enable);

/* Reset the counters and record only the phases whose bit (1u << SVT_PH_*) is set in mask;
 * mask = 0 stops recording.  Errors: SVT_E_INVALID_ARG (bits above SVT_PH_COUNT). */
svt_status svt_profile_phases(svt_handle* h, uint32_t mask);

/* Benchmark support: `reps` back-to-back launches of the kernel of one single-kernel phase
 * (SVT_PH_SPMM_T, SVT_PH_GRAM, SVT_PH_SDDMM or SVT_PH_DENSIFY) on the operands the last iteration
 * left, between two hipEvents on the handle's stream.  Events around launches inside the
 * iteration also count the time the GPU waits for the host to enqueue the kernel after a host
 * decision point; here the launches queue behind each other, so the per-launch time is the
 * kernel's own plus the dispatch gap between consecutive kernels.
 * Outputs: *ms = device milliseconds per launch; *bytes, *flops (may be NULL) = algorithmic work
 * of one launch (as svt_profile_read counts it).  The replayed kernels rewrite only buffers that
 * every iteration rewrites before reading them (W, G, the dense copy of Y, the next Y and the
 * partial sums), so the iteration state is unchanged.
 * Errors: SVT_E_INVALID_ARG (another phase, reps < 1, ms == NULL), SVT_E_STATE (no iteration
 * run yet, or the phase has no kernel in this problem). */
svt_status svt_time_phase(svt_handle* h, int32_t phase, int32_t reps, double* ms, double* bytes, double* flops);

/* Per phase (arrays of SVT_PH_COUNT entries, any may be NULL): device milliseconds, algorithmic
 * bytes moved (each operand counted once per launch), algorithmic flops, number of launches. */
svt_status svt_profile_read(svt_handle* h, double* ms, double* bytes, double* flops, int64_t* launches);

/* Text of the last error on this handle (or of the last failed svt_init when h is NULL). */
const char* svt_last_error(const svt_handle* h);

/* Wait for the handle's stream (svt_iterate may return with the next step's
 * first kernels still queued), then release every device and host buffer of
 * the handle.  NULL is allowed. */
void svt_destroy(svt_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* SVT_H */
