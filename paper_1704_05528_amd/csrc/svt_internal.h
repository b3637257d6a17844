// Internal declarations shared by the device kernels and the host control of libsvt.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/svt.h"

namespace svt {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per workgroup for streaming kernels
constexpr int kEigMax = 96;        // largest Rayleigh-Ritz block the in-LDS Jacobi solver holds
constexpr int kNarrow = 16;        // widest block handled by the lanes-over-nonzeros SpMM
constexpr int kScalars = 64;       // doubles in the device->host readback buffer

// Device buffers of one problem.  Matrices are row-major; "ld" is the row stride.
struct Handle {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t m = 0, n = 0, nnz = 0;
  svt_params p{};
  int32_t r_cap = 0;      // columns allocated for Q and W (>= r_max)
  int32_t w_cap = 0;      // columns allocated for a sampled block (>= max(t0, dt))
  int32_t b_cap = 0;      // columns of the eigensolver block (kEigMax)

  // sparsity structure
  int32_t *colptr = nullptr, *rowidx = nullptr;   // CSC (primary order of values)
  int32_t *rowptr = nullptr, *colidx = nullptr;   // CSR
  int32_t *csr2csc = nullptr;                     // CSR position -> CSC position
  int32_t *tstart = nullptr;                      // row-tile starts per column (dense-ish patterns only)
  std::vector<int64_t> user2csc;                  // caller order -> CSC position (host)

  // values on Lambda (CSC order)
  double *a = nullptr, *y = nullptr, *y_next = nullptr, *x = nullptr;

  // basis and projections
  double *Q = nullptr;    // m x r_cap
  double *W = nullptr;    // n x r_cap, W = Y^T Q = B^T
  double *X = nullptr;    // m x w_cap sampled block
  double *X2 = nullptr;   // m x w_cap scratch block
  double *Om = nullptr;   // n x w_cap Gaussian block, also Y^T X scratch for power iterations
  double *T = nullptr;    // r_cap x w_cap projection coefficients Q^T X
  double *G = nullptr;    // r_cap x r_cap Gram W^T W
  double *small = nullptr;  // w_cap x w_cap Gram / factor scratch
  double *Minv = nullptr;   // w_cap x w_cap orthonormalising transform
  double *prenorm = nullptr;  // w_cap column norms before projection

  // eigensolver
  double *EV = nullptr, *EZ = nullptr, *EZ2 = nullptr, *EZ3 = nullptr;  // r_cap x kEigMax blocks
  double *EH = nullptr, *ES = nullptr;                  // b_cap x b_cap Rayleigh quotient and its eigvecs
  double *Eval = nullptr;                               // b_cap eigenvalues (descending)
  int32_t ev_valid = 0;   // columns of EV that hold Ritz vectors of the previous iteration
  int32_t ev_rows = 0;    // basis width those vectors refer to

  // factors of X = Ut Vt^T
  double *Ut = nullptr;   // m x kEigMax, Q U_K diag(sigma - tau)
  double *Vt = nullptr;   // n x kEigMax, W U_K diag(1 / sigma)
  double *C = nullptr;    // r_cap x kEigMax
  double *D = nullptr;    // r_cap x kEigMax
  double *Sk = nullptr;   // r_cap x kEigMax, eigenvectors of the Gram for sigma > tau
  double *Utmp = nullptr; // max(m, n) x kEigMax scratch
  int32_t k = 0;
  std::vector<double> sigma_k;   // host copy of the k singular values above tau

  // reductions
  double *partial = nullptr;  int64_t partial_cap = 0;
  double *scal = nullptr;     // device scalars
  double *hscal = nullptr;    // pinned host mirror

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
  std::vector<int32_t> replay_blocks, replay_anneal;
  size_t replay_pos = 0;

  // instrumentation: hipEvent pairs per phase, resolved at the next host synchronisation
  struct Pending {
    int ph;
    hipEvent_t e0, e1;
  };
  bool prof = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  double ph_ms[SVT_PH_COUNT] = {};
  double ph_bytes[SVT_PH_COUNT] = {};
  double ph_flops[SVT_PH_COUNT] = {};
  int64_t ph_launch[SVT_PH_COUNT] = {};

  std::string err;
};

// ---------------------------------------------------------------------------------------------
// kernel launchers (kernels.hip)
// ---------------------------------------------------------------------------------------------
// columns c0 .. c0+w-1 (c0 a multiple of 4) of the Omega block (it, blk), stored from column 0 of om
hipError_t launch_omega(hipStream_t s, double* om, int n, int c0, int w, int ld, uint64_t seed, uint64_t blk,
                        uint64_t it);

// out[row, 0:w] = sum over the row's segment of val[vperm ? vperm[p] : p] * D[idx[p], 0:w]
hipError_t launch_seg_spmm(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* vperm,
                           const double* val, const double* D, int ldd, double* out, int ldo, int w);

// columns c0 .. c0+count-1 of a rows x ld block set to e_{row0}, e_{row0+1}, ...
hipError_t launch_set_unit(hipStream_t s, double* V, int rows, int ld, int c0, int count, int row0);

// LDS-tiled W = Y^T Q for densely sampled patterns; tstart holds, for every column j, the CSC
// position of its first entry in each row tile (n x (tiled_row_tiles(m) + 1) int32)
int tiled_row_tiles(int64_t m);
hipError_t launch_spmm_t_tiled(hipStream_t s, int m, int n, const int32_t* rowidx, const int32_t* tstart,
                               const double* val, const double* Q, int ldq, int r, double* W, int ldw,
                               double* partial, int64_t partial_cap);

// out[i, 0:w] = beta * out[i, 0:w] + alpha * A[i, 0:K] M[0:K, 0:w]
hipError_t launch_rowmul(hipStream_t s, int rows, int K, const double* A, int lda, const double* M, int ldm,
                         double* out, int ldo, int w, double alpha, double beta);

// partial Gram blocks: out[a, b] = sum_i A[i, a] B[i, b], a < na (any), b < nb (<= 64)
hipError_t launch_tn_narrow(hipStream_t s, int rows, const double* A, int lda, int na, const double* B, int ldb,
                            int nb, double* out, int ldo, double* partial, int64_t partial_cap);

// Gram G = A^T A for A rows x na (na up to r_cap), full symmetric output
hipError_t launch_gram(hipStream_t s, int rows, const double* A, int lda, int na, double* G, int ldg,
                       double* partial, int64_t partial_cap);

// scal[slot] = sum of squares over the columns c0..c0+w-1 of a rows x ld matrix
hipError_t launch_sumsq_cols(hipStream_t s, int rows, const double* A, int lda, int c0, int w, double* partial,
                             double* scal, int slot);
// scal[slot] = sum v[i]^2
hipError_t launch_sumsq(hipStream_t s, int64_t len, const double* v, double* partial, double* scal, int slot);
// out[c] = ||A[:, c]||_2 for c < w (w <= 64), via the w x w Gram in gram_scratch
hipError_t launch_colnorms(hipStream_t s, int rows, const double* A, int lda, int w, double* gram_scratch,
                           double* partial, int64_t partial_cap, double* out);

// Cholesky factor R of a block's Gram with the column-drop rules (one workgroup): see kernels.hip
hipError_t launch_block_chol(hipStream_t s, const double* gram, int ldg, int w, const double* prenorm,
                             double drop_tol, double dep_tol, double* Rout, int ldm, double* scal, int slot,
                             int wk_slot_in);
// out = X[:, kept] R^{-1} row by row, kept columns packed left, the rest zero
hipError_t launch_trsm_rows(hipStream_t s, int rows, const double* X, int ldx, int w, const double* R, int ldr,
                           double* out, int ldo);

// sampled product on Lambda (CSC order) with residual and dual update; per-block partial sums of
// res^2 and y_next^2 land in partial[2 b], partial[2 b + 1]; returns the number of blocks
hipError_t launch_sddmm_update(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx, const double* a,
                               const double* y, double* y_next, double* x_out, const double* Ut, const double* Vt,
                               int ld, int k, double delta, double* partial, int* nblocks);
// scal[slot + q] = sum_b partial[b * stride + q], q < nq, in block order
hipError_t launch_finish(hipStream_t s, const double* partial, int nblocks, int stride, int nq, double* scal, int slot);
// X on arbitrary entries
hipError_t launch_sample(hipStream_t s, int64_t nq, const int32_t* qi, const int32_t* qj, const double* Ut,
                         const double* Vt, int ld, int k, double* out);

hipError_t launch_scale_copy(hipStream_t s, int64_t len, const double* src, double alpha, double* dst);
hipError_t launch_copy_cols(hipStream_t s, int rows, const double* src, int lds, double* dst, int ldd, int w);

// ---------------------------------------------------------------------------------------------
// eigensolver (eig.hip)
// ---------------------------------------------------------------------------------------------
// Jacobi eigen-decomposition of a b x b symmetric matrix (b <= kEigMax) in one workgroup.
// Eigenvalues descending into eval, eigenvectors as columns of evec (row-major, ld = ldv).
hipError_t launch_jacobi(hipStream_t s, const double* H, int ldh, int b, double* eval, double* evec, int ldv,
                         double* scal, int slot, int max_sweeps = 40);
// residual column norms ||Z[:, c] - theta_c V[:, c]|| for c < b
hipError_t launch_ritz_residual(hipStream_t s, int rows, const double* Z, const double* V, int ld, int b,
                                const double* theta, double* partial, double* out);
// factor matrices C = S[:, :k] diag(sigma - tau), D = S[:, :k] diag(1/sigma) from eigenpairs of the Gram
hipError_t launch_factor_coeffs(hipStream_t s, int r, int k, const double* S, int lds, const double* theta,
                                double tau, double* C, double* D, int ldc);
// fill columns c0..c1-1 of an r x ld block with Philox Gaussians (rows >= r zero)
hipError_t launch_fill_random(hipStream_t s, double* V, int rows, int ld, int c0, int c1, uint64_t seed,
                              uint64_t tag);

}  // namespace svt
