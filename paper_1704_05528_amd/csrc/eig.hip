// Symmetric eigen-solver pieces for the small projected SVD of R4SVD (Alg. 3, svd(B)).
//
// svd(B) of the r x n matrix B = Q^T Y is taken through the Gram matrix
// G = B B^T = W^T W (r x r, float64): eig(G) = U_B diag(sigma^2) U_B^T.  Only the
// eigenpairs with sigma > tau enter D_tau (Eq. 5).  When r fits one workgroup the whole
// G is diagonalised by cyclic Jacobi; otherwise a warm-started block subspace iteration
// (host control in svt_api.hip) reduces G to a b x b Rayleigh quotient that this Jacobi
// kernel diagonalises.
#include "svt_internal.h"

namespace svt {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Cyclic Jacobi (Golub & Van Loan, sym.schur2 rotations) with round-robin ordering: in each
// round the bb/2 disjoint pairs rotate at once.  With J block-diagonal over the pairs, every
// 2 x 2 block (P, R) of J^T A J depends only on the same block of A, so one pass over the
// blocks applies the round (rows and columns together), and V <- V J in the same pass.
// A and V live in LDS.  Sweeps stop when the off-diagonal mass is below 1e-30 of the total
// squared Frobenius norm, or after max_sweeps.
__global__ __launch_bounds__(256) void k_jacobi(const double* __restrict__ H, int ldh, int b,
                                                double* __restrict__ eval, double* __restrict__ evec, int ldv,
                                                double* scal, int slot, int max_sweeps) {
  extern __shared__ double sm[];
  const int bb = b + (b & 1);
  const int ld = bb + 1;
  double* A = sm;
  double* V = sm + bb * ld;
  __shared__ double cs[kEigMax / 2], sn[kEigMax / 2];
  __shared__ int pp[kEigMax / 2], qq[kEigMax / 2];
  __shared__ double red[8];
  __shared__ int perm[kEigMax];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wid = tid / kWave;
  const int half = bb / 2;

  for (int e = tid; e < bb * bb; e += blockDim.x) {
    const int i = e / bb, j = e % bb;
    A[i * ld + j] = (i < b && j < b) ? 0.5 * (H[(int64_t)i * ldh + j] + H[(int64_t)j * ldh + i]) : 0.0;
    V[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  // A rotation is skipped when |a_pq| <= eps sqrt(|a_pp a_qq|) (the relative test of Demmel and
  // Veselic for positive semidefinite matrices) or when |a_pq| is below 1e-19 of the largest
  // diagonal entry (irrelevant at working precision); a sweep without any rotation ends it.
  __shared__ int rotated;
  __shared__ double dmax_s;
  if (tid == 0) {
    double d = 0.0;
    for (int i = 0; i < b; ++i) d = fmax(d, fabs(A[i * ld + i]));
    dmax_s = d;
  }
  __syncthreads();
  const double dmax = dmax_s;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < bb - 1; ++round) {
      if (tid < half) {
        const int t = tid;
        const int pa = (t == 0) ? 0 : 1 + ((t - 1 + round) % (bb - 1));
        const int pb = 1 + ((bb - 2 - t + round) % (bb - 1));
        const int p = min(pa, pb), q = max(pa, pb);
        const double apq = A[p * ld + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0 && fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(A[p * ld + p] * A[q * ld + q])) &&
            fabs(apq) > 1e-19 * dmax) {
          rotated = 1;
          const double app = A[p * ld + p], aqq = A[q * ld + q];
          const double th = (aqq - app) / (2.0 * apq);
          double tt;
          if (fabs(th) > 1e150) {
            tt = 0.5 / th;
          } else {
            tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
          }
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        cs[t] = c;
        sn[t] = s;
        pp[t] = p;
        qq[t] = q;
      }
      __syncthreads();
      // blocks (P, R): rows p1, q1 rotate by pair P, columns p2, q2 by pair R
      for (int e = tid; e < half * half; e += blockDim.x) {
        const int P = e / half, R = e % half;
        const int p1 = pp[P], q1 = qq[P], p2 = pp[R], q2 = qq[R];
        const double c1 = cs[P], s1 = sn[P], c2 = cs[R], s2 = sn[R];
        const double a00 = A[p1 * ld + p2], a01 = A[p1 * ld + q2];
        const double a10 = A[q1 * ld + p2], a11 = A[q1 * ld + q2];
        const double r00 = c1 * a00 - s1 * a10, r01 = c1 * a01 - s1 * a11;
        const double r10 = s1 * a00 + c1 * a10, r11 = s1 * a01 + c1 * a11;
        A[p1 * ld + p2] = c2 * r00 - s2 * r01;
        A[p1 * ld + q2] = s2 * r00 + c2 * r01;
        A[q1 * ld + p2] = c2 * r10 - s2 * r11;
        A[q1 * ld + q2] = s2 * r10 + c2 * r11;
      }
      for (int e = tid; e < bb * half; e += blockDim.x) {
        const int i = e / half, R = e % half;
        const int p = pp[R], q = qq[R];
        const double c = cs[R], s = sn[R];
        const double vp = V[i * ld + p], vq = V[i * ld + q];
        V[i * ld + p] = c * vp - s * vq;
        V[i * ld + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();   // every thread has read the flag before thread 0 clears it again
    if (!any) break;
  }

  // sort eigenvalues descending (the padding index of odd b has eigenvalue 0 and is excluded)
  if (tid == 0) {
    for (int i = 0; i < b; ++i) perm[i] = i;
    for (int i = 0; i < b; ++i) {
      int best = i;
      for (int j = i + 1; j < b; ++j)
        if (A[perm[j] * ld + perm[j]] > A[perm[best] * ld + perm[best]]) best = j;
      const int t = perm[i];
      perm[i] = perm[best];
      perm[best] = t;
    }
    scal[slot] = (double)sweep;
  }
  __syncthreads();
  for (int i = tid; i < b; i += blockDim.x) eval[i] = A[perm[i] * ld + perm[i]];
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int i = e / b, c = e % b;
    evec[(int64_t)i * ldv + c] = V[i * ld + perm[c]];
  }
}

// res[c] = || Z[:, c] - theta[c] V[:, c] ||_2, one workgroup per column (deterministic).
__global__ __launch_bounds__(256) void k_ritz_residual(int rows, const double* __restrict__ Z,
                                                       const double* __restrict__ V, int ld,
                                                       const double* __restrict__ theta, double* __restrict__ out) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  const double th = theta[c];
  double acc = 0.0;
  for (int i = threadIdx.x; i < rows; i += blockDim.x) {
    const double d = Z[(int64_t)i * ld + c] - th * V[(int64_t)i * ld + c];
    acc = fma(d, d, acc);
  }
  acc = wave_sum(acc);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = sqrt(((red[0] + red[1]) + red[2]) + red[3]);
}

// C[:, c] = S[:, c] (sigma_c - tau), D[:, c] = S[:, c] / sigma_c, sigma_c = sqrt(theta_c), c < k.
__global__ void k_factor_coeffs(int r, int k, const double* __restrict__ S, int lds_, const double* __restrict__ theta,
                                double tau, double* __restrict__ C, double* __restrict__ D, int ldc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)r * k) return;
  const int i = (int)(t / k), c = (int)(t % k);
  const double sg = sqrt(theta[c]);
  const double v = S[(int64_t)i * lds_ + c];
  C[(int64_t)i * ldc + c] = v * (sg - tau);
  D[(int64_t)i * ldc + c] = v / sg;
}

}  // namespace

hipError_t launch_jacobi(hipStream_t s, const double* H, int ldh, int b, double* eval, double* evec, int ldv,
                         double* scal, int slot, int max_sweeps) {
  const int bb = b + (b & 1);
  const size_t lds = (size_t)2 * bb * (bb + 1) * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((size_t)2 * kEigMax * (kEigMax + 1) * sizeof(double)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), lds, s, H, ldh, b, eval, evec, ldv, scal, slot, max_sweeps);
  return hipGetLastError();
}

hipError_t launch_ritz_residual(hipStream_t s, int rows, const double* Z, const double* V, int ld, int b,
                                const double* theta, double* partial, double* out) {
  (void)partial;
  if (b == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ritz_residual, dim3(b), dim3(256), 0, s, rows, Z, V, ld, theta, out);
  return hipGetLastError();
}

hipError_t launch_factor_coeffs(hipStream_t s, int r, int k, const double* S, int lds_, const double* theta,
                                double tau, double* C, double* D, int ldc) {
  const int64_t work = (int64_t)r * k;
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL(k_factor_coeffs, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, r, k, S, lds_, theta,
                     tau, C, D, ldc);
  return hipGetLastError();
}

}  // namespace svt
