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

// One workgroup, double.  U: r x r eigenvectors of G (columns, descending eigenvalues theta),
// Z1 = Bbar V_K (r x k), Z2 = Bbar B^T (r x r).  Writes Cmat (r x (2k + r), ld ldc) and
// scal[slot] = tau_bar; scratch: r x r (ld r) in global memory.  LDS: 4 r k + r doubles.
__global__ __launch_bounds__(256) void k_adjoint_coeffs(int r, int k, const double* __restrict__ U, int ldu,
                                                        const double* __restrict__ theta,
                                                        const double* __restrict__ Z1, int ldz1,
                                                        const double* __restrict__ Z2, int ldz2, double tau,
                                                        double* __restrict__ Cmat, int ldc, double* __restrict__ scratch,
                                                        double* scal, int slot) {
  extern __shared__ double sm[];
  double* M1 = sm;                      // r x k : U^T Bbar V_K
  double* M2 = M1 + r * k;              // k x r : U_K^T Bbar B^T U
  double* T2 = M2 + k * r;              // k x r : U_K^T Z2, then r x k : coefficient matrix Ec
  double* Bt = T2 + k * r;              // r x k : Beta (rows j in N)
  double* sg = Bt + r * k;              // r singular values
  __shared__ double lds[4];
  const int tid = threadIdx.x;
  for (int j = tid; j < r; j += blockDim.x) sg[j] = sqrt(fmax(theta[j], 0.0));
  for (int e = tid; e < r * k; e += blockDim.x) {
    const int j = e / k, c = e % k;
    double v = 0.0;
    for (int l = 0; l < r; ++l) v = fma(U[(int64_t)l * ldu + j], Z1[(int64_t)l * ldz1 + c], v);
    M1[j * k + c] = v;
  }
  for (int e = tid; e < k * r; e += blockDim.x) {
    const int c = e / r, j = e % r;
    double v = 0.0;
    for (int l = 0; l < r; ++l) v = fma(U[(int64_t)l * ldu + c], Z2[(int64_t)l * ldz2 + j], v);
    T2[c * r + j] = v;
  }
  __syncthreads();
  for (int e = tid; e < k * r; e += blockDim.x) {
    const int c = e / r, j = e % r;
    double v = 0.0;
    for (int l = 0; l < r; ++l) v = fma(T2[c * r + l], U[(int64_t)l * ldu + j], v);
    M2[c * r + j] = v;
  }
  __syncthreads();
  double tr = 0.0;
  for (int c = tid; c < k; c += blockDim.x) tr += M1[c * k + c];
  const double trs = block_sum(tr, lds);
  if (tid == 0) scal[slot] = -trs;
  // Ec[i][c]: Gamma_ic for i in K, Kappa_ic for i in N; Beta[j][i] for j in N (zero for j in K)
  double* Ec = T2;
  for (int e = tid; e < r * k; e += blockDim.x) {
    const int i = e / k, c = e % k;
    const double sc = sg[c], fc = sc - tau;
    double v;
    if (i < k) {
      const double si = sg[i], fi = si - tau;
      if (i == c) {
        v = M1[i * k + c] - fi / si * M1[i * k + c];
      } else {
        const double a = (si != sc) ? (fi - fc) / (si - sc) : 1.0;
        const double b = (fi + fc) / (si + sc);
        v = 0.5 * (a + b) * M1[i * k + c] + 0.5 * (a - b) * M1[c * k + i] - fi / si * M1[i * k + c];
      }
    } else {
      const double si = sg[i];
      v = fc * (sc * M1[i * k + c] + M2[c * r + i]) / (sc * sc - si * si);
    }
    Ec[i * k + c] = v;
    // Beta[j = i][c]  (the role of the K index is played by c here)
    double bt = 0.0;
    if (i >= k) {
      const double sj = sg[i];
      bt = (fc / sc * M2[c * r + i] + fc * M1[i * k + c]) / (sc * sc - sj * sj);
    }
    Bt[i * k + c] = bt;
  }
  __syncthreads();
  // Cmat[:, 0:k] = U_K diag(f/s);  Cmat[:, k:2k] = U Ec;  scratch = U_K Beta^T (r x r)
  for (int e = tid; e < r * k; e += blockDim.x) {
    const int l = e / k, c = e % k;
    const double sc = sg[c];
    Cmat[(int64_t)l * ldc + c] = U[(int64_t)l * ldu + c] * (sc - tau) / sc;
    double v = 0.0;
    for (int i = 0; i < r; ++i) v = fma(U[(int64_t)l * ldu + i], Ec[i * k + c], v);
    Cmat[(int64_t)l * ldc + k + c] = v;
  }
  for (int e = tid; e < r * r; e += blockDim.x) {
    const int l = e / r, j = e % r;
    double v = 0.0;
    for (int i = 0; i < k; ++i) v = fma(U[(int64_t)l * ldu + i], Bt[j * k + i], v);
    scratch[(int64_t)l * r + j] = v;
  }
  __threadfence_block();
  __syncthreads();
  // Cmat[:, 2k:2k+r] = (U_K Beta^T) U^T
  for (int e = tid; e < r * r; e += blockDim.x) {
    const int l = e / r, q = e % r;
    double v = 0.0;
    for (int j = k; j < r; ++j) v = fma(scratch[(int64_t)l * r + j], U[(int64_t)q * ldu + j], v);
    Cmat[(int64_t)l * ldc + 2 * k + q] = v;
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
  constexpr int kMaxLds = 160 * 1024 - 256;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_adjoint_coeffs, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kMaxLds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const size_t lds = (size_t)(4 * r * std::max(k, 1) + r) * sizeof(double);
  if (lds > (size_t)kMaxLds) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adjoint_coeffs, dim3(1), dim3(256), lds, s, r, k, U, ldu, theta, Z1, ldz1, Z2, ldz2, tau, Cmat,
                     ldc, scratch, scal, slot);
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
