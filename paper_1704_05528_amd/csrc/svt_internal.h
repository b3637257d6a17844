// Internal declarations shared by the device kernels and the host control of libsvt.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include <string>
#include <vector>

#include "../../include/svt.h"

namespace svt {

constexpr int kWave = 64;     // CDNA wavefront width
constexpr int64_t kKPartElems = (int64_t)256 * 64 * 48;  // a product split over K: at most 256 tiles of 64 x 48
constexpr int kEigMax = 96;   // largest block the in-LDS Jacobi / Cholesky kernels hold
constexpr int kEB = 1024;     // widest block of the subspace eigen-solver (columns of EV, EZ, ES)
constexpr int kNarrow = 16;   // widest block handled by the lanes-over-nonzeros SpMM
constexpr int kScalars = 64;  // doubles in the device->host readback buffer
constexpr int kSpecSlot = 48;  // host slot of the next iteration's ||W||^2 (past every readback's range)
constexpr int kStageDoubles = 4096;  // pinned staging doubles for small device->host copies
constexpr int kSddmmChunk = 256;  // most CSC positions one wave of the fused sampled update takes

// bfloat16 storage (the basis of the BF16 form): the upper half of a float32.  Conversion from
// float rounds to nearest, ties to even; conversion to float is exact.
struct bf16 {
  uint16_t bits;
  bf16() = default;
  __host__ __device__ explicit bf16(float f) : bits(round(f)) {}
  __host__ __device__ explicit bf16(double d) : bits(round((float)d)) {}
  __host__ __device__ explicit bf16(int i) : bits(round((float)i)) {}
  __host__ __device__ operator float() const { return __builtin_bit_cast(float, (uint32_t)bits << 16); }
  __host__ __device__ static uint16_t round(float f) {
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays a (quiet) NaN
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  }
};
static_assert(sizeof(bf16) == 2, "bf16 is two bytes");

// Newton-Raphson refinement (two steps each, quadratic convergence from the hardware estimates)
// of the double reciprocal and reciprocal square root: short dependent chains for the small
// one-workgroup factorisations, where an IEEE division sits on the critical path.
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}
__device__ inline double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

// ------------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and Box-Muller: the Gaussian sampling matrix Omega of
// Alg. 2 / Alg. 3.  Counter = (row j, 4-column group q, block, iteration), key = (seed, 0).
// ------------------------------------------------------------------------------------------
__device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

__device__ inline double word_to_uniform(uint64_t w) {
  return ((double)(w >> 11) + 0.5) * 0x1p-53;
}

__device__ inline void gaussian4(uint64_t j, uint64_t q, uint64_t blk, uint64_t it, uint64_t seed, double z[4]) {
  uint64_t c[4] = {j, q, blk, it};
  philox4x64_10(c, seed, 0ull);
#pragma unroll
  for (int pr = 0; pr < 2; ++pr) {
    const double ur = word_to_uniform(c[2 * pr]), ua = word_to_uniform(c[2 * pr + 1]);
    const double rad = sqrt(-2.0 * log(ur));
    const double ang = 2.0 * M_PI * ua;
    z[2 * pr] = rad * cos(ang);
    z[2 * pr + 1] = rad * sin(ang);
  }
}

// Copies src[0..count) to mapped host memory and then sets *flag = seq, with every value visible to
// the host first (each thread's system-scope fence, the barrier, then thread 0's); one workgroup.
// The source may have been written by this workgroup before the call.
__device__ inline void post_to_host(const double* src, int count, double* dst, unsigned* flag, unsigned seq) {
  __threadfence_block();
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = src[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    *(volatile unsigned*)flag = seq;
  }
}

// sum_{t < n} p[t * stride] in a fixed order (16 interleaved partial sums, then a fixed tree),
// with 16 independent loads in flight: the split sums of the tall products are latency bound
// when each load waits for the previous add.
template <class T>
__device__ inline T split_sum(const T* __restrict__ p, int n, int64_t stride) {
  constexpr int kU = 16;
  T acc[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) acc[u] = (T)0;
  for (int t0 = 0; t0 < n; t0 += kU) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u;
      const T x = p[(int64_t)min(t, n - 1) * stride];
      acc[u] += (t < n) ? x : (T)0;
    }
  }
#pragma unroll
  for (int o = kU / 2; o > 0; o >>= 1)
#pragma unroll
    for (int u = 0; u < o; ++u) acc[u] += acc[u + o];
  return acc[0];
}

// Long segments of a segment-gather product cut into chunks (device arrays): chunk q covers
// positions [lo[q], hi[q]); long segment t = lcol[t] owns chunks lfirst[t] .. lfirst[t+1]-1;
// skip[row] != 0 marks the rows the chunked form computes; P holds nchunk partial rows of ldp
// values of the storage type.
struct SegChunks {
  int32_t nlong = 0, nchunk = 0, ldp = 0;
  int32_t *lo = nullptr, *hi = nullptr, *lcol = nullptr, *lfirst = nullptr, *skip = nullptr;
  void* P = nullptr;
};
constexpr int kSegLong = 256;  // a segment longer than this is cut into chunks of this many positions

// Device buffers of one problem.  Matrices are row-major; "ld" is the row stride.  Buffers
// marked (T) hold the storage type of the precision form: double (SVT_FP64) or float
// (SVT_MIXED); the Gram matrices, the eigensolver and all reductions are double in both.
struct Handle {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t m = 0, n = 0, nnz = 0;
  svt_params p{};
  int32_t r_cap = 0;  // columns allocated for Q and W (>= r_max + 64)
  int32_t w_cap = 0;  // columns of a sampled block chunk (64)
  int32_t b_cap = 0;  // columns of the eigensolver block

  // sparsity structure
  int32_t *colptr = nullptr, *rowidx = nullptr;  // CSC (primary order of values)
  int32_t *rowptr = nullptr, *colidx = nullptr;  // CSR
  int32_t *csr2csc = nullptr;                    // CSR position -> CSC position
  int32_t *tstart = nullptr;                     // row-tile starts per column (dense-ish patterns only)
  int32_t *cstart = nullptr, *ccol = nullptr;    // load-balanced chunks of the CSC order (fused update)
  void* yT = nullptr;  // (T) n x m dense transposed copy of Y (zeros off Lambda) when >= 25% is observed
  int32_t nchunks = 0;
  int32_t max_row_nnz = 0, max_col_nnz = 0;  // longest row / column of Lambda (picks the gather's launch shape)
  SegChunks csc_long;  // long columns of Y for W = Y^T D on the sparse path
  std::vector<int64_t> user2csc;                 // caller order -> CSC position (host)

  // values on Lambda, CSC order (T)
  void *a = nullptr, *y = nullptr, *y_next = nullptr;

  // basis, projections, sampled blocks (T)
  void* Q = nullptr;   // m x r_cap
  void* W = nullptr;   // n x r_cap, W = Y^T Q = B^T
  void* X = nullptr;   // m x w_cap sampled block
  void* X2 = nullptr;  // m x w_cap scratch block
  void* Om = nullptr;  // max(m, n) x w_cap Gaussian block, also Y^T X in power iterations
  // double
  double* T = nullptr;        // r_cap x w_cap projection coefficients Q^T X
  double* G = nullptr;        // r_cap x r_cap Gram W^T W
  double* G2 = nullptr;       // r_cap x r_cap, G^2 for the double steps of the block eigensolver
  double* small = nullptr;    // kEigMax x kEigMax block Gram
  double* Minv = nullptr;     // kEigMax x kEigMax block Cholesky factor
  double* prenorm = nullptr;  // column norms before projection

  // eigensolver (double)
  double *EV = nullptr, *EZ = nullptr, *EZ2 = nullptr, *EZ3 = nullptr;  // r_cap x kEB blocks
  double *EH = nullptr, *ES = nullptr;                                   // kEB x kEB
  double* Eval = nullptr;  // eigenvalues (descending) followed by Ritz residual norms
  int32_t ev_valid = 0;    // columns of EV that hold Ritz vectors of the previous iteration
  int32_t ev_rows = 0;     // basis width those vectors refer to
  int32_t eig_pred = 6;    // products with G before the first Rayleigh-Ritz test (adapted each iteration)
  int32_t eig_pass_streak = 0;  // consecutive iterations whose first test passed
  double cheb_c = 0.0;  // smallest Ritz value of the last accepted block (0: none): the damped interval of the filter

  // full eigen-decomposition of G (Jacobi over many workgroups, eigfull.hip), used once the count
  // above tau outgrows the block solver; r_cap x r_cap matrices allocated on first use
  bool full_mode = false;   // the projected SVD diagonalises all of G (sticky while k stays large)
  int32_t fe_rows = 0;      // leading rows / columns of FEt, FEU that hold the last full solve's vectors
  double *JA = nullptr, *JV = nullptr, *FM = nullptr;  // Jacobi matrix, its rotations (rows), product scratch
  double *FEt = nullptr, *FEU = nullptr;              // eigenvectors of G as rows / as columns, descending
  double *Fval = nullptr, *Jpin = nullptr, *Jtol = nullptr, *Jpart = nullptr;
  int32_t *Jperm = nullptr, *Jflag = nullptr;

  // factors of X = Ut Vt^T; ldf columns each (the most singular values above tau tracked)
  int32_t ldf = 0;
  void* Ut = nullptr;      // (T) m x ldf, Q S_K diag(sigma - tau)
  void* Vt = nullptr;      // (T) n x ldf, W S_K diag(1 / sigma)
  void* Utmp = nullptr;    // (T) max(m, n) x ldf scratch
  double* C = nullptr;     // r_cap x ldf
  double* D = nullptr;     // r_cap x ldf
  double* Sk = nullptr;    // r_cap x ldf, eigenvectors of the Gram for sigma > tau

  // BF16 form: inverse Cholesky factor of the stored basis's Gram Q^T Q (lower, r_cap x r_cap), its
  // transpose, and scratch for the bordering steps
  double *Linv = nullptr, *LinvT = nullptr, *Lw = nullptr, *Lw2 = nullptr;
  bool gp_valid = false;  // the leading work left the corrected Gram of the current basis in G
  bool gp_now = false;    // G holds it within the current R4SVD call
  int32_t k = 0;
  std::vector<double> sigma_k;  // host copy of the k singular values above tau

  // reductions
  double* partial = nullptr;
  int64_t partial_cap = 0;
  double* kpart = nullptr;  // K-split partial products of the dense W = Y^T Q (kKPartElems doubles)
  double* scal = nullptr;   // device scalars
  double* hscal = nullptr;  // pinned host mirror (mapped into the device: hscal_d)
  double* hstage = nullptr; // pinned staging area of kStageDoubles doubles for small readbacks (hstage_d)
  double* hscal_d = nullptr;
  double* hstage_d = nullptr;
  unsigned* hflag = nullptr;    // mapped host word: the sequence number of the last completed post
  unsigned* hflag_d = nullptr;
  unsigned post_seq = 0;        // sequence number of the last post enqueued
  unsigned spec_seq = 0;        // the post that carries the next iteration's ||W||^2
  unsigned sync_seq = 0;        // the post that carries an iteration's sums
  double* scratch = nullptr;  // this device's copy of the library's file-scope scratch array (svt_mae_device)
  hipEvent_t sync_ev = nullptr;  // timing-free event the host spins on at decision points
  // The next iteration's leading work (dense copy of Y, W = Y^T Q, ||W||^2) was enqueued at the end
  // of the previous iteration; ||W||^2 lands in hscal[kSpecSlot] when post spec_seq completes.
  bool spec_ready = false;
  hipEvent_t spec_ev = nullptr;

  // iteration state (host)
  int32_t r = 0;
  int32_t iter = 0;
  double eps_thr = 0.0;
  bool eps_thr_set = false;
  double eps_min = 0.0;
  double normY = 0.0;
  double norm_a = 0.0;
  int32_t k0 = 0;
  bool converged = false;
  bool have_factors = false;
  bool lost = false;      // a wait for the device timed out: its buffers may still be in use
  bool ready = false;     // svt_init has finished (the caller's wait limit applies from then on)
  int32_t div_run = 0;    // iterations in a row with the residual above 10 times its minimum
  std::vector<int32_t> replay_blocks, replay_anneal;
  size_t replay_pos = 0;
  // basis width used by every iteration since svt_init (the basis only grows, so the basis of
  // iteration i is the first hist_r[i] columns of Q); svt_set_state invalidates it
  std::vector<int32_t> hist_r;
  bool hist_ok = true;
  // every sampled chunk appended to the basis since svt_init, in order: SVT iteration (1-based),
  // Omega block, its first column and width, and the basis column it starts at.  exact_ok: no chunk
  // lost a column and no power iteration ran, so the basis is the plain chain the exact reverse
  // sweep differentiates.
  struct ChunkRec {
    int32_t it, blk, c0, w, q0;
  };
  std::vector<ChunkRec> hist_chunks, cur_chunks;
  bool exact_ok = true;

  // instrumentation: hipEvent pairs per phase, resolved at the next host synchronisation
  struct Pending {
    int ph;
    hipEvent_t e0, e1;
  };
  uint32_t prof_mask = 0;  // phases recorded by the phase timers (bit 1 << SVT_PH_*)
  std::vector<svt_step_stats> history;  // reports of the iterations run by svt_iterate
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  double ph_ms[SVT_PH_COUNT] = {};
  double ph_bytes[SVT_PH_COUNT] = {};
  double ph_flops[SVT_PH_COUNT] = {};
  int64_t ph_launch[SVT_PH_COUNT] = {};

  std::string err;
};

// ---------------------------------------------------------------------------------------------
// kernel launchers (kernels.hip); T is double or float
// ---------------------------------------------------------------------------------------------
// columns c0 .. c0+w-1 (c0 a multiple of 4) of the Omega block (it, blk), stored from column 0 of om
template <class T>
hipError_t launch_omega(hipStream_t s, T* om, int n, int c0, int w, int ld, uint64_t seed, uint64_t blk, uint64_t it);


// out[row, 0:w] = sum over the row's segment of val[vperm ? vperm[p] : p] * D[idx[p], 0:w].  total is
// the number of positions in all segments and max_len the longest segment (they pick the launch
// shape only).  With ch, the long
// segments (over kSegLong positions) run as kSegLong chunks spread over the chip, their partial
// sums in ch->P, instead of on one wave each.
constexpr int kNarrowSplitLen = 256;   // narrow blocks: a workgroup per segment from this mean length on,
constexpr int kNarrowSplitMax = 1024;  // or from this longest segment on
template <class T, class TD>
hipError_t launch_seg_spmm(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* vperm,
                           const T* val, const TD* D, int ldd, T* out, int ldo, int w, int64_t total, int max_len,
                           const SegChunks* ch = nullptr);

// LDS-tiled W = Y^T Q for densely sampled patterns; tstart holds, for every column j, the CSC
// position of its first entry in each row tile (n x (tiled_row_tiles(m) + 1) int32)
int tiled_row_tiles(int64_t m);
template <class T, class TQ>
hipError_t launch_spmm_t_tiled(hipStream_t s, int m, int n, const int32_t* rowidx, const int32_t* tstart,
                               const T* val, const TQ* Q, int ldq, int r, T* W, int ldw, double* partial,
                               int64_t partial_cap);

// One product of launch_rowmul / launch_rowmul_pair (see below)
template <class TA, class TM, class TO>
struct RowmulProblem {
  int rows, K;
  const TA* A;
  int lda;
  const TM* M;
  int ldm;
  TO* out;
  int ldo, w;
  double alpha, beta;
  double* gpart;
};

// out[i, 0:w] = beta * out[i, 0:w] + alpha * A[i, 0:K] M[0:K, 0:w] (double accumulation).  With gpart
// (w <= 16 only): gpart[t][a][b] (t = 16-row tile, w x w each) = the Gram of the tile's stored rows.
template <class TA, class TM, class TO>
hipError_t launch_rowmul(hipStream_t s, int rows, int K, const TA* A, int lda, const TM* M, int ldm, TO* out, int ldo,
                         int w, double alpha, double beta, double* gpart = nullptr);
// two independent products of launch_rowmul in one launch (they run side by side)
template <class TA, class TM, class TO>
hipError_t launch_rowmul_pair(hipStream_t s, const RowmulProblem<TA, TM, TO>& p0, const RowmulProblem<TA, TM, TO>& p1);

// out[a * ldo + b] = sum over s < splits of partial[s * na * nb + a * nb + b] (fixed order)
hipError_t launch_tn_finish(hipStream_t s, const double* partial, int splits, int na, int nb, double* out, int ldo);

// out[a, b] = sum_i A[i, a] B[i, b] in double, a < na (any), b < nb (<= kEigMax)
template <class TA, class TB>
hipError_t launch_tn_narrow(hipStream_t s, int rows, const TA* A, int lda, int na, const TB* B, int ldb, int nb,
                            double* out, int ldo, double* partial, int64_t partial_cap);

// The sum of squares of a product's output, taken by the kernel that writes it as per-workgroup
// partials: partial[0..*nparts) (at most cap of them), to be added by launch_finish.
struct NormReq {
  double* partial = nullptr;
  int64_t cap = 0;
};

// dense C = A B (row-major) on the matrix cores in the storage precision (float or double accumulation);
// B may be stored in bfloat16 for float (widened on load).  tri = 1: A is lower triangular, tri = 2: B is
// upper triangular (the zero parts are not read).  With a workspace of work_elems elements a product
// with few output tiles is also split over K (partial products there, then added in a fixed order).
// With nrm, a product split over K also leaves the partial sums of squares of C (see NormReq) from the
// kernel that adds the parts, and *nparts is their count (0 when it did not: the caller takes them).
template <class T, class TB>
hipError_t launch_gemm_nn(hipStream_t s, int M, int N, int K, const T* A, int lda, const TB* B, int ldb, T* C, int ldc,
                          int tri = 0, T* work = nullptr, int64_t work_elems = 0, const NormReq* nrm = nullptr,
                          int* nparts = nullptr);
// G = A^T A (A rows x na row-major, G na x na double) from 64 x 64 tiles staged in LDS on the
// matrix cores; gram_tn_tiles(na) is the number of workgroups it launches.  launch_gram takes it
// from rows * na >= kGramTiledMin on.
constexpr int64_t kGramTiledMin = 40'000'000;
template <class T>
hipError_t launch_gram_tn(hipStream_t s, int rows, const T* A, int lda, int na, double* G, int ldg);
int gram_tn_tiles(int na);
// yT[j * ldy + i] = y(i, j) on Lambda (the other entries of yT are left untouched)
template <class T>
hipError_t launch_scatter_dense_t(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx, const T* y, T* yT,
                                  int64_t ldy);
// Gram G = A^T A in double for A rows x na (na up to r_cap), full symmetric output
template <class T>
hipError_t launch_gram(hipStream_t s, int rows, const T* A, int lda, int na, double* G, int ldg, double* partial,
                       int64_t partial_cap);

// A device -> host post attached to the kernel that produces the values (see launch_post): after its
// own work the kernel copies src[0..count) to dst (mapped host memory) and sets *flag = seq.
struct PostReq {
  const double* src = nullptr;
  int count = 0;
  double* dst = nullptr;
  unsigned* flag = nullptr;
  unsigned seq = 0;
};

// scal[slot] = sum of squares over the columns c0..c0+w-1 of a rows x ld matrix (then the post, if any)
template <class T>
hipError_t launch_sumsq_cols(hipStream_t s, int rows, const T* A, int lda, int c0, int w, double* partial,
                             double* scal, int slot, const PostReq* post = nullptr);
// scal[slot] = sum v[i]^2
template <class T>
hipError_t launch_sumsq(hipStream_t s, int64_t len, const T* v, double* partial, double* scal, int slot);
// out[c] = ||A[:, c]||_2 for c < w (w <= 64), via the w x w Gram in gram_scratch
template <class T>
hipError_t launch_colnorms(hipStream_t s, int rows, const T* A, int lda, int w, double* gram_scratch, double* partial,
                           int64_t partial_cap, double* out);

// Cholesky factor R of a block's Gram with the column-drop rules (one workgroup): see kernels.hip
// The Gram may be given as the sum of `splits` partial Grams sstride doubles apart.
hipError_t launch_block_chol(hipStream_t s, const double* gram, int ldg, int w, const double* prenorm,
                             double drop_tol, double dep_tol, double* Rout, int ldm, double* scal, int slot,
                             int wk_slot_in, int splits = 1, int64_t sstride = 0);
// partial[s][a][b] of A^T B split over rows, without the final sum; *splits_out receives the split
// count (the consumer adds the splits, stride na * nb)
template <class TA, class TB>
hipError_t launch_tn_partial(hipStream_t s, int rows, const TA* A, int lda, int na, const TB* B, int ldb, int nb,
                             double* partial, int64_t partial_cap, int* splits_out);
// out = X[:, kept] R^{-1} row by row, kept columns packed left, the rest zero
template <class T>
hipError_t launch_trsm_rows(hipStream_t s, int rows, const T* X, int ldx, int w, const double* R, int ldr, T* out,
                            int ldo);

// One CholeskyQR pass out = X[:, kept] R^{-1} from the Gram partials of X (splits matrices w x w,
// sstride apart) in one launch of one-wave workgroups of 64 rows, each factoring the Gram itself
// (k_block_chol's drop rules: prenorm / drop_tol, dep_tol; wk_slot_in >= 0 limits the columns to
// scal[wk_slot_in]).  gout (may be NULL): the Gram partials of out, one w x w matrix per 64 rows.
// scal[slot] = kept count.  w <= kCholTrsmMaxCols; hipErrorInvalidValue otherwise.
constexpr int kCholTrsmMaxCols = 96;
constexpr int kCholTrsmMaxRows = 4096;  // above this a separate factor launch costs less than the repeats
template <class T>
hipError_t launch_chol_trsm(hipStream_t s, int rows, const T* X, int ldx, int w, const double* gram, int splits,
                            int64_t sstride, const double* prenorm, double drop_tol, double dep_tol, int wk_slot_in,
                            T* out, int ldo, double* gout, double* scal, int slot);

// sampled product on Lambda (CSC order) with residual and dual update, one wave per chunk of at
// most kSddmmChunk positions of one column (chunk c = [cstart[c], cstart[c+1]) in column ccol[c]);
// per-block partial sums of res^2, y_next^2 and |res| land in partial[3 b], partial[3 b + 1],
// partial[3 b + 2]; *nblocks receives the block count.  With yT non-null, y_next at position
// (i, j) is also stored to yT[j * ldy + i] (the dense transposed copy; other entries untouched).
template <class T>
hipError_t launch_sddmm_update(hipStream_t s, int nchunks, const int32_t* cstart, const int32_t* ccol,
                               const int32_t* rowidx, const T* a, const T* y, T* y_next, const T* Ut, const T* Vt,
                               int ld, int k, double delta, double* partial, int* nblocks, T* yT = nullptr,
                               int64_t ldy = 0);
// scal[slot + q] = sum_b partial[b * stride + q], q < nq, in block order (then the post, if any)
hipError_t launch_finish(hipStream_t s, const double* partial, int nblocks, int stride, int nq, double* scal, int slot,
                         const PostReq* post = nullptr);
// Copies count doubles to host memory mapped into the device (dst_mapped: its device address) and then
// sets the mapped flag to seq: the host polls the flag instead of waiting for a copy and an event.
hipError_t launch_post(hipStream_t s, const double* src, int count, double* dst_mapped, unsigned* flag_mapped,
                       unsigned seq);
// scal[slot] = sum |ref - x| over len entries (deterministic)
hipError_t launch_absdiff_sum(hipStream_t s, int64_t len, const double* x, const double* ref, double* partial,
                              double* scal, int slot);
// MAE of X against ref on nq entries in one pass without storing X: work holds kMaeFusedBlocks
// partial sums and their total (kMaeFusedBlocks + 1 doubles); out[0] = total / nq.  Same value as
// launch_sample followed by launch_absdiff_sum.
constexpr int kMaeFusedBlocks = 1024;
template <class T>
hipError_t launch_mae_fused(hipStream_t s, int64_t nq, const int32_t* qi, const int32_t* qj, const T* Ut, const T* Vt,
                           int ld, int k, int64_t m, int64_t n, const double* ref, double* work, double* out);
// X on arbitrary entries; an index outside m x n gives NaN
template <class T>
hipError_t launch_sample(hipStream_t s, int64_t nq, const int32_t* qi, const int32_t* qj, const T* Ut, const T* Vt,
                         int ld, int k, int64_t m, int64_t n, double* out);

template <class TS, class TD>
hipError_t launch_scale_copy(hipStream_t s, int64_t len, const TS* src, double alpha, TD* dst);
template <class TS, class TD>
hipError_t launch_copy_cols(hipStream_t s, int rows, const TS* src, int lds, TD* dst, int ldd, int w);
// BF16 form: the bordering step of the inverse Cholesky factor Linv of the stored basis's Gram
// (w <= 64 appended columns at rq; Gq22 = Q'^T Q', P = L21 L21^T or nullptr when rq = 0); writes
// Linv22 and its transpose, clears the strips above / left of them, scal[slot] = 1 on a pivot
// that is not positive
hipError_t launch_border_chol(hipStream_t s, const double* Gq22, int ldg, const double* P, int ldp, int w, int rq,
                              double* Linv, double* LinvT, int ld, double* scal, int slot);
// scal[slot] = trace(G[0:r, 0:r])
hipError_t launch_trace(hipStream_t s, const double* G, int ld, int r, double* scal, int slot);

// dst[t] = src[perm[t]], t < len
hipError_t launch_gather_perm(hipStream_t s, int64_t len, const int32_t* perm, const double* src, double* dst);

// columns c0 .. c0+count-1 of a rows x ld block set to e_{row0}, e_{row0+1}, ...
hipError_t launch_set_unit(hipStream_t s, double* V, int rows, int ld, int c0, int count, int row0);
// fill columns c0..c1-1 of a rows x ld block with Philox Gaussians
hipError_t launch_fill_random(hipStream_t s, double* V, int rows, int ld, int c0, int c1, uint64_t seed,
                              uint64_t tag);

// ---------------------------------------------------------------------------------------------
// eigensolver (eig.hip), double
// ---------------------------------------------------------------------------------------------
// The block subspace iteration (npairs double steps with CholeskyQR) and its Rayleigh-Ritz step for a
// basis of r <= kSmallR columns and a block of b <= kSmallB, in one workgroup (G and the block in LDS).
// EV (r x b, ld ldv) holds the start block on entry and the Ritz vectors on exit, GV gets G times them,
// eval[0..b) the Ritz values (descending) and eval[ldres + c] the residual norms.
constexpr int kSmallR = 112, kSmallB = 16;
// Columns valid .. b-1 of the start block are drawn in the kernel (launch_fill_random's values for seed and
// tag) and rows ev_rows .. r-1 of the first valid columns read as zero, so the block needs no set-up launch.
// With post_dst given, the b Ritz values and then the b residual norms are also written there (mapped
// host memory) and *post_flag set to post_seq.
hipError_t launch_eig_small(hipStream_t s, int r, const double* G, int ldg, double* EV, double* GV, int ldv, int b,
                            int npairs, bool filt, double alpha, double beta, double dep_tol, double* eval, int ldres,
                            double* scal, int slot, int max_sweeps, int valid, int ev_rows, uint64_t seed,
                            uint64_t tag, double* post_dst = nullptr, unsigned* post_flag = nullptr,
                            unsigned post_seq = 0);

// P = alpha P + beta G + I on the leading r x r blocks (ld) of two symmetric matrices
hipError_t launch_cheb2(hipStream_t s, int r, double* P, const double* G, int ld, double alpha, double beta);

// Jacobi eigen-decomposition of a b x b symmetric matrix (b <= kEigMax) in one workgroup.
// Eigenvalues descending into eval, eigenvectors as columns of evec (row-major, ld = ldv).
// H may be given as the sum of `splits` matrices sstride doubles apart (split partial products).
hipError_t launch_jacobi(hipStream_t s, const double* H, int ldh, int b, double* eval, double* evec, int ldv,
                         double* scal, int slot, int max_sweeps = 40, int splits = 1, int64_t sstride = 0);
// residual column norms ||Z[:, c] - theta_c V[:, c]|| for c < b
hipError_t launch_ritz_residual(hipStream_t s, int rows, const double* Z, const double* V, int ld, int b,
                                const double* theta, double* partial, double* out);
// factor matrices C = S[:, :k] diag(sigma - tau), D = S[:, :k] diag(1/sigma) from eigenpairs of the Gram,
// and zeros in their columns k .. kpad-1 (kpad >= k; 0 means k)
hipError_t launch_factor_coeffs(hipStream_t s, int r, int k, const double* S, int lds, const double* theta,
                                double tau, double* C, double* D, int ldc, double* Sk = nullptr, int kpad = 0);

// ---------------------------------------------------------------------------------------------
// full eigen-decomposition (eigfull.hip), double: cyclic Jacobi over many workgroups, one launch
// per round-robin round
// ---------------------------------------------------------------------------------------------
constexpr int kJgMaxOrder = 4096;  // largest matrix order (slots per workgroup stay <= 8)
constexpr int kJgMaxWg = 256;      // workgroups per round before a workgroup takes several slots
// Pads an odd n with a zero row and column (A, ld lda >= n + 1), sets Vt = I (nn x nn) when
// vt_identity (otherwise only its padding), writes the rotation inputs of round 0 into pin (3 nn / 2
// doubles) and the rotation threshold (1e-15 of the largest diagonal entry) into *tolp.
hipError_t launch_jg_start(hipStream_t s, double* A, int lda, int n, double* Vt, int ldv, bool vt_identity,
                           double* pin, double* tolp);
// One round rd (0 <= rd < nn - 1, nn even) in place on A and the rows of Vt; pin_cur / pin_next:
// this round's and the next round's rotation inputs; *flag = 1 when a pair rotates.
hipError_t launch_jg_round(hipStream_t s, double* A, int lda, double* Vt, int ldv, int nn, int rd, const double* pin_cur,
                           double* pin_next, const double* tolp, int32_t* flag);
// out[0] = max_{i < j} |A_ij| (part: 256 doubles), out[1] = the threshold
hipError_t launch_jg_offmax(hipStream_t s, const double* A, int lda, int nn, const double* tolp, double* part,
                            double* out);
// eigenvalues descending (ties by index) into eval, eigenvector c as row c of Et and column c of EU
// (either may be NULL); perm: n ints
hipError_t launch_jg_finish(hipStream_t s, const double* A, int lda, const double* Vt, int ldv, int n, int32_t* perm,
                            double* eval, double* Et, int ldet, double* EU, int ldeu);
// M[i][j] = delta_ij outside the leading r0 x r0 block of the r x r matrix M
hipError_t launch_extend_identity(hipStream_t s, double* M, int ld, int r0, int r);
// dst (cols x rows) = src^T (src rows x cols)
hipError_t launch_transpose(hipStream_t s, const double* src, int lds_, int rows, int cols, double* dst, int ldd);

// ---------------------------------------------------------------------------------------------
// reverse sweep (adjoint.hip), double
// ---------------------------------------------------------------------------------------------
// Cmat = [U_K diag(f/s) | U_K Gamma + U_N Kappa | U_K Beta^T U^T] (r x (2k + r)) and scal[slot] =
// tau_bar for one unrolled iteration; U, theta: full eigen-decomposition of G, Z1 = Bbar V_K (r x k),
// Z2 = Bbar B^T (r x r); scratch: adjoint_coeffs_scratch(r, k) doubles.  1 <= k <= r.
// Adjoint of a thin QR with R of positive diagonal, for one w x w block (w <= 64, one workgroup):
// C = copyltu(-M) (the symmetric matrix with the lower triangle of -M) and RinvT = R^{-T} (R the
// upper triangle of Rm).  All w x w with row stride ld.
hipError_t launch_qr_adjoint_coeffs(hipStream_t s, int w, const double* Rm, const double* M, double* C, double* RinvT,
                                    int ld);
hipError_t launch_adjoint_coeffs(hipStream_t s, int r, int k, const double* U, int ldu, const double* theta,
                                 const double* Z1, int ldz1, const double* Z2, int ldz2, double tau, double* Cmat,
                                 int ldc, double* scratch, double* scal, int slot);
size_t adjoint_coeffs_scratch(int r, int k);
// out[p] = <L[row(p), 0:w], R[col(p), 0:w]> on Lambda (CSC order)
hipError_t launch_lambda_dot(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx, const double* L,
                             int ldl, const double* R, int ldr, int w, double* out);
// res = a - x, y_next = y + delta res
hipError_t launch_dual_update(hipStream_t s, int64_t nnz, const double* a, const double* x, const double* y,
                              double delta, double* res, double* y_next);
// dst = alpha x + beta dst
hipError_t launch_axpby(hipStream_t s, int64_t len, double alpha, const double* x, double beta, double* dst);
// scal[slot] = <x, y> (deterministic)
hipError_t launch_dot(hipStream_t s, int64_t len, const double* x, const double* y, double* partial, double* scal,
                      int slot);

}  // namespace svt
