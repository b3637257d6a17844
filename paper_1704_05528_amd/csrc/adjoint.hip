// Device pieces of the reverse sweep through unrolled SVT iterations (frozen-basis convention).
//
// Iteration i maps Y_i to X_i = Q_i D_tau(B_i), B_i = Q_i^T Y_i, with the basis and every discrete
// decision held fixed.  For a cotangent Xbar on X_i, with Bbar = Q_i^T Xbar, the eigenpairs
// (theta_j = sigma_j^2, u_j) of G = B B^T, K = {sigma_j > tau}, f_j = sigma_j - tau on K, and
// V_K = B^T U_K diag(1/sigma_K), the adjoint Bbar -> dB of the thresholding map (derivative of
// spectral functions of rectangular matrices) can be written without the singular vectors of
// the small singular values:
//   dB = U_K diag(f/s) P^T + (U_K Gamma + U_N Kappa) V_K^T + U_K Beta^T U^T B
// with P = Bbar^T U_K, M1 = U^T Bbar V_K, M2 = U_K^T Bbar B^T U and, for i, c in K, j in N:
//   Gamma_ic = (a+b)/2 M1_ic + (a-b)/2 M1_ci - f_i/s_i M1_ic  (i != c),  Gamma_ii = M1_ii - f_i/s_i M1_ii,
//   a = (f_i - f_c)/(s_i - s_c),  b = (f_i + f_c)/(s_i + s_c),
//   Kappa_jc = f_c (s_c M1_jc + M2_cj) / (s_c^2 - s_j^2),
//   Beta_ji  = (f_i/s_i M2_ij + f_i M1_ji) / (s_i^2 - s_j^2).
// The sampled adjoint Ybar = P_Lambda(Q dB) is then one sampled product with the factor pair
//   L = Q [U_K diag(f/s) | U_K Gamma + U_N Kappa | U_K Beta^T U^T],  R = [P | V_K | W],  W = B^T.
// tau_bar = -trace(M1_KK).
#include "svt_internal.h"

#include <algorithm>

namespace svt {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += lds[i];
  return t;
}

// The coefficient block of one unrolled iteration, in global memory (any r), as five grid-wide
// passes with one thread per output entry.  U: r x r eigenvectors of G (columns, descending
// eigenvalues theta), Z1 = Bbar V_K (r x k), Z2 = Bbar B^T (r x r).  Work arrays (ld as noted):
// M1 = U^T Z1 (r x k), T2 = U_K^T Z2 (k x r), M2 = T2 U (k x r), Ec (r x k), Bt (r x k), S = U_K Bt^T
// (r x r).  Cmat = [U_K diag(f/s) | U Ec | S U^T restricted to j in N] (r x (2k + r), ld ldc).
struct AdjWork {
  double *M1, *T2, *M2, *Ec, *Bt, *S;
};

__device__ inline double sg_of(const double* theta, int j) { return sqrt(fmax(theta[j], 0.0)); }

__global__ void k_adj_m1t2(int r, int k, const double* __restrict__ U, int ldu, const double* __restrict__ Z1, int ldz1,
                           const double* __restrict__ Z2, int ldz2, AdjWork w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rk = (int64_t)r * k;
  if (e < rk) {
    const int j = (int)(e / k), c = (int)(e % k);
    double v = 0.0;
    for (int l = 0; l < r; ++l) v = fma(U[(int64_t)l * ldu + j], Z1[(int64_t)l * ldz1 + c], v);
    w.M1[j * (int64_t)k + c] = v;
  } else if (e < 2 * rk) {
    const int64_t f = e - rk;
    const int c = (int)(f / r), j = (int)(f % r);
    double v = 0.0;
    for (int l = 0; l < r; ++l) v = fma(U[(int64_t)l * ldu + c], Z2[(int64_t)l * ldz2 + j], v);
    w.T2[c * (int64_t)r + j] = v;
  }
}

__global__ void k_adj_m2(int r, int k, const double* __restrict__ U, int ldu, AdjWork w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * r) return;
  const int c = (int)(e / r), j = (int)(e % r);
  double v = 0.0;
  for (int l = 0; l < r; ++l) v = fma(w.T2[c * (int64_t)r + l], U[(int64_t)l * ldu + j], v);
  w.M2[c * (int64_t)r + j] = v;
}

// tau_bar = -trace(M1_KK) in the order of one 256-thread block sum
__global__ __launch_bounds__(256) void k_adj_trace(int k, AdjWork w, double* scal, int slot) {
  __shared__ double lds[4];
  double tr = 0.0;
  for (int c = threadIdx.x; c < k; c += blockDim.x) tr += w.M1[c * (int64_t)k + c];
  const double trs = block_sum(tr, lds);
  if (threadIdx.x == 0) scal[slot] = -trs;
}

// Ec[i][c]: Gamma_ic for i in K, Kappa_ic for i in N; Bt[j][c] = Beta_jc for j in N (zero in K);
// Cmat[:, c] = U_K diag(f/s) for c < k
__global__ void k_adj_coeffs(int r, int k, const double* __restrict__ U, int ldu, const double* __restrict__ theta,
                             double tau, AdjWork w, double* __restrict__ Cmat, int ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * k) return;
  const int i = (int)(e / k), c = (int)(e % k);
  const double* M1 = w.M1;
  const double* M2 = w.M2;
  const double sc = sg_of(theta, c), fc = sc - tau;
  double v;
  if (i < k) {
    const double si = sg_of(theta, i), fi = si - tau;
    if (i == c) {
      v = M1[i * (int64_t)k + c] - fi / si * M1[i * (int64_t)k + c];
    } else {
      const double a = (si != sc) ? (fi - fc) / (si - sc) : 1.0;
      const double b = (fi + fc) / (si + sc);
      v = 0.5 * (a + b) * M1[i * (int64_t)k + c] + 0.5 * (a - b) * M1[c * (int64_t)k + i] - fi / si * M1[i * (int64_t)k + c];
    }
  } else {
    const double si = sg_of(theta, i);
    v = fc * (sc * M1[i * (int64_t)k + c] + M2[c * (int64_t)r + i]) / (sc * sc - si * si);
  }
  w.Ec[i * (int64_t)k + c] = v;
  double bt = 0.0;
  if (i >= k) {
    const double sj = sg_of(theta, i);
    bt = (fc / sc * M2[c * (int64_t)r + i] + fc * M1[i * (int64_t)k + c]) / (sc * sc - sj * sj);
  }
  w.Bt[i * (int64_t)k + c] = bt;
  // Cmat[:, 0:k]: row i of U_K diag(f/s) (i plays the row index l here)
  Cmat[(int64_t)i * ldc + c] = U[(int64_t)i * ldu + c] * (sc - tau) / sc;
}

// Cmat[:, k:2k] = U Ec and S = U_K Bt^T (r x r)
__global__ void k_adj_uec(int r, int k, const double* __restrict__ U, int ldu, AdjWork w, double* __restrict__ Cmat,
                          int ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rk = (int64_t)r * k;
  if (e < rk) {
    const int l = (int)(e / k), c = (int)(e % k);
    double v = 0.0;
    for (int i = 0; i < r; ++i) v = fma(U[(int64_t)l * ldu + i], w.Ec[i * (int64_t)k + c], v);
    Cmat[(int64_t)l * ldc + k + c] = v;
  } else if (e < rk + (int64_t)r * r) {
    const int64_t f = e - rk;
    const int l = (int)(f / r), j = (int)(f % r);
    double v = 0.0;
    for (int i = 0; i < k; ++i) v = fma(U[(int64_t)l * ldu + i], w.Bt[j * (int64_t)k + i], v);
    w.S[(int64_t)l * r + j] = v;
  }
}

// Cmat[:, 2k:2k+r] = S U^T over the columns j in N
__global__ void k_adj_sut(int r, int k, const double* __restrict__ U, int ldu, AdjWork w, double* __restrict__ Cmat,
                          int ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int l = (int)(e / r), q = (int)(e % r);
  double v = 0.0;
  for (int j = k; j < r; ++j) v = fma(w.S[(int64_t)l * r + j], U[(int64_t)q * ldu + j], v);
  Cmat[(int64_t)l * ldc + 2 * k + q] = v;
}

// C = copyltu(-M), RinvT = R^{-T}: one thread per column c of R^{-1}, by back substitution on the
// upper triangle of Rm (z_i = (delta_ic - sum_{j > i} R_ij z_j) / R_ii for i = c .. 0).
__global__ __launch_bounds__(64) void k_qr_adjoint_coeffs(int w, const double* __restrict__ Rm,
                                                          const double* __restrict__ M, double* __restrict__ C,
                                                          double* __restrict__ RinvT, int ld) {
  __shared__ double R[64][65];
  const int t = threadIdx.x;
  for (int e = t; e < w * w; e += 64) {
    const int i = e / w, j = e % w;
    R[i][j] = (j >= i) ? Rm[i * ld + j] : 0.0;
    const int a = max(i, j), b = min(i, j);
    C[i * ld + j] = -M[a * ld + b];
  }
  __syncthreads();
  if (t < w) {
    double z[64];
    for (int i = w - 1; i >= 0; --i) {
      double v = (i == t) ? 1.0 : 0.0;
      for (int j = i + 1; j < w; ++j) v -= R[i][j] * ((j <= t) ? z[j] : 0.0);
      z[i] = (i <= t) ? v / R[i][i] : 0.0;
    }
    for (int i = 0; i < w; ++i) RinvT[t * ld + i] = z[i];
  }
}

// out[p] = sum_l L[row(p), l] R[col(p), l] for the CSC positions p of Lambda (one thread each)
__global__ void k_lambda_dot(int n, const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                             const double* __restrict__ L, int ldl, const double* __restrict__ R, int ldr, int w,
                             double* __restrict__ out) {
  const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (j >= n) return;
  const double* rr = R + (int64_t)j * ldr;
  for (int p = colptr[j] + lane; p < colptr[j + 1]; p += kWave) {
    const double* ll = L + (int64_t)rowidx[p] * ldl;
    double v = 0.0;
    for (int l = 0; l < w; ++l) v = fma(ll[l], rr[l], v);
    out[p] = v;
  }
}

// res = a - x; y_next = y + delta res (double, elementwise)
__global__ void k_dual_update(int64_t nnz, const double* __restrict__ a, const double* __restrict__ x,
                              const double* __restrict__ y, double delta, double* __restrict__ res,
                              double* __restrict__ y_next) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const double rv = a[p] - x[p];
  res[p] = rv;
  y_next[p] = fma(delta, rv, y[p]);
}

// dst = alpha * x + beta * dst
__global__ void k_axpby(int64_t len, double alpha, const double* __restrict__ x, double beta, double* __restrict__ dst) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= len) return;
  dst[p] = alpha * x[p] + (beta == 0.0 ? 0.0 : beta * dst[p]);
}

__global__ __launch_bounds__(256) void k_dot(int64_t len, const double* __restrict__ x, const double* __restrict__ y,
                                             double* __restrict__ partial) {
  __shared__ double lds[4];
  double v = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x)
    v = fma(x[e], y[e], v);
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

inline unsigned grid1(int64_t work, int per = 256) { return (unsigned)((work + per - 1) / per); }

}  // namespace

hipError_t launch_adjoint_coeffs(hipStream_t s, int r, int k, const double* U, int ldu, const double* theta,
                                 const double* Z1, int ldz1, const double* Z2, int ldz2, double tau, double* Cmat,
                                 int ldc, double* scratch, double* scal, int slot) {
  if (r <= 0 || k <= 0 || k > r) return hipErrorInvalidValue;
  const int64_t rk = (int64_t)r * k, rr = (int64_t)r * r;
  AdjWork w;
  w.M1 = scratch;
  w.T2 = w.M1 + rk;
  w.M2 = w.T2 + rk;
  w.Ec = w.M2 + rk;
  w.Bt = w.Ec + rk;
  w.S = w.Bt + rk;
  hipLaunchKernelGGL(k_adj_m1t2, dim3(grid1(2 * rk)), dim3(256), 0, s, r, k, U, ldu, Z1, ldz1, Z2, ldz2, w);
  hipLaunchKernelGGL(k_adj_m2, dim3(grid1(rk)), dim3(256), 0, s, r, k, U, ldu, w);
  hipLaunchKernelGGL(k_adj_trace, dim3(1), dim3(256), 0, s, k, w, scal, slot);
  hipLaunchKernelGGL(k_adj_coeffs, dim3(grid1(rk)), dim3(256), 0, s, r, k, U, ldu, theta, tau, w, Cmat, ldc);
  hipLaunchKernelGGL(k_adj_uec, dim3(grid1(rk + rr)), dim3(256), 0, s, r, k, U, ldu, w, Cmat, ldc);
  hipLaunchKernelGGL(k_adj_sut, dim3(grid1(rr)), dim3(256), 0, s, r, k, U, ldu, w, Cmat, ldc);
  return hipGetLastError();
}

size_t adjoint_coeffs_scratch(int r, int k) { return (size_t)5 * r * k + (size_t)r * r; }

hipError_t launch_qr_adjoint_coeffs(hipStream_t s, int w, const double* Rm, const double* M, double* C, double* RinvT,
                                    int ld) {
  if (w <= 0 || w > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_qr_adjoint_coeffs, dim3(1), dim3(64), 0, s, w, Rm, M, C, RinvT, ld);
  return hipGetLastError();
}

hipError_t launch_lambda_dot(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx, const double* L,
                             int ldl, const double* R, int ldr, int w, double* out) {
  hipLaunchKernelGGL(k_lambda_dot, dim3((n + 3) / 4), dim3(256), 0, s, n, colptr, rowidx, L, ldl, R, ldr, w, out);
  return hipGetLastError();
}

hipError_t launch_dual_update(hipStream_t s, int64_t nnz, const double* a, const double* x, const double* y,
                              double delta, double* res, double* y_next) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dual_update, dim3(grid1(nnz)), dim3(256), 0, s, nnz, a, x, y, delta, res, y_next);
  return hipGetLastError();
}

hipError_t launch_axpby(hipStream_t s, int64_t len, double alpha, const double* x, double beta, double* dst) {
  if (len == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby, dim3(grid1(len)), dim3(256), 0, s, len, alpha, x, beta, dst);
  return hipGetLastError();
}

hipError_t launch_dot(hipStream_t s, int64_t len, const double* x, const double* y, double* partial, double* scal,
                      int slot) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (len + 255) / 256));
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(256), 0, s, len, x, y, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finish(s, partial, nb, 1, 1, scal, slot);
}

}  // namespace svt
