// Symmetric eigen-solver pieces for the small projected SVD of R4SVD (Alg. 3, svd(B)).
//
// svd(B) of the r x n matrix B = Q^T Y is taken through the Gram matrix
// G = B B^T = W^T W (r x r, float64): eig(G) = U_B diag(sigma^2) U_B^T.  Only the
// eigenpairs with sigma > tau enter D_tau (Eq. 5).  When r fits one workgroup the whole
// G is diagonalised by cyclic Jacobi; otherwise a warm-started block subspace iteration
// (host control in svt_api.hip) reduces G to a b x b Rayleigh quotient that this Jacobi
// kernel diagonalises.
#include "svt_internal.h"

#include <algorithm>

namespace svt {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}


constexpr int kHalfMax = kEigMax / 2;

// Cyclic Jacobi (Golub & Van Loan, sym.schur2 rotations) with round-robin ordering: in each
// round the bb/2 disjoint pairs rotate at once.  With J block-diagonal over the pairs, every
// 2 x 2 block (P, R) of J^T A J depends only on the same block of A, so one pass over the
// blocks applies the round (rows and columns together), and V <- V J in the same pass.
// A and V live in LDS.  A pair rotates when |a_pq| exceeds 1e-15 of the largest diagonal entry
// (absolute accuracy, which is what the top eigenpairs need); a sweep without any rotation
// ends the iteration.  The rotating threads all sit in wave 0, so one ballot decides whether a
// round rotates at all.  Each thread gathers the operands of its blocks before updating them
// (its blocks never overlap), so one round costs two LDS round trips per thread.
__global__ __launch_bounds__(256) void k_jacobi(const double* __restrict__ H, int ldh, int splits, int64_t sstride,
                                                int b, double* __restrict__ eval, double* __restrict__ evec,
                                                int ldv, double* scal, int slot, int max_sweeps) {
  constexpr int CA = 3, CV = 5;  // blocks of A and row pairs of V per thread and chunk
  extern __shared__ double sm[];
  const int bb = b + (b & 1);
  const int ld = bb + 1;
  const int half = bb / 2;
  const float inv_half = 1.0f / (float)half;
  double* A = sm;
  double* V = sm + bb * ld;
  __shared__ double cs[kHalfMax], sn[kHalfMax];
  __shared__ int pp[kHalfMax], qq[kHalfMax];
  __shared__ double red[4];
  __shared__ int flag[2];
  __shared__ int rank_of[kEigMax];
  const int tid = threadIdx.x;

  // H is the sum of `splits` matrices sstride apart (partial products, added in a fixed order)
  for (int e = tid; e < bb * bb; e += blockDim.x) {
    const int i = e / bb, j = e - (e / bb) * bb;
    double hij = 0.0, hji = 0.0;
    if (i < b && j < b) {
      hij = split_sum(H + (int64_t)i * ldh + j, splits, sstride);
      hji = split_sum(H + (int64_t)j * ldh + i, splits, sstride);
    }
    A[i * ld + j] = 0.5 * (hij + hji);
    V[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double dm = 0.0;
  for (int i = tid; i < b; i += blockDim.x) dm = fmax(dm, fabs(A[i * ld + i]));
  dm = fmax(dm, __shfl_xor(dm, 32, kWave));
  dm = fmax(dm, __shfl_xor(dm, 16, kWave));
  dm = fmax(dm, __shfl_xor(dm, 8, kWave));
  dm = fmax(dm, __shfl_xor(dm, 4, kWave));
  dm = fmax(dm, __shfl_xor(dm, 2, kWave));
  dm = fmax(dm, __shfl_xor(dm, 1, kWave));
  if ((tid & (kWave - 1)) == 0) red[tid / kWave] = dm;
  __syncthreads();
  const double tol = 1e-15 * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const int nb1 = bb - 1;
  const int totA = half * half, totV = bb * half;
  int sweep = 0, seq = 0;  // seq: rounds since the start; its parity picks the flag, so a wave
                           // that sets the next round's flag never overwrites one still being read
  for (; sweep < max_sweeps; ++sweep) {
    int sweep_any = 0;
    for (int round = 0; round < nb1; ++round, ++seq) {
      int mine = 0;
      if (tid < half) {
        // round-robin pairing: slot 0 fixed, the others rotate by one position per round
        const int t = tid;
        int x = t - 1 + round;
        x = (x >= nb1) ? x - nb1 : x;
        int y = bb - 2 - t + round;
        y = (y >= nb1) ? y - nb1 : y;
        const int pa = (t == 0) ? 0 : 1 + x;
        const int pb = 1 + y;
        const int p = min(pa, pb), q = max(pa, pb);
        const double apq = A[p * ld + q], app = A[p * ld + p], aqq = A[q * ld + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > tol) {
          mine = 1;
          // tangent of the smaller rotation angle that annihilates a_pq
          const double dd = aqq - app;
          const double den = fabs(dd) + sqrt(fma(dd, dd, 4.0 * apq * apq));
          const double tt = (dd >= 0.0 ? 2.0 : -2.0) * apq * rcp_nr(den);
          c = rsq_nr(fma(tt, tt, 1.0));
          s = tt * c;
        }
        cs[t] = c;
        sn[t] = s;
        pp[t] = p;
        qq[t] = q;
      }
      if (tid < kWave) {
        const unsigned long long bal = __ballot(mine);
        if (tid == 0) flag[seq & 1] = (bal != 0ull);
      }
      __syncthreads();
      if (!flag[seq & 1]) continue;  // uniform: nothing rotates, nothing to update this round
      sweep_any = 1;
      if (bb <= 32) {
        // small blocks: one pass over the 2 x 2 blocks of A and the row pairs of V, no chunking
        // (at these sizes the gather-then-update chunks below cost more than they save)
        for (int e = tid; e < totA + totV; e += blockDim.x) {
          if (e < totA) {
            const int P = e / half, R = e - (e / half) * half;
            const int p1 = pp[P], q1 = qq[P], p2 = pp[R], q2 = qq[R];
            const double c1 = cs[P], s1 = sn[P], c2 = cs[R], s2 = sn[R];
            const double a0 = A[p1 * ld + p2], a1 = A[p1 * ld + q2], a2 = A[q1 * ld + p2], a3 = A[q1 * ld + q2];
            const double r00 = c1 * a0 - s1 * a2, r01 = c1 * a1 - s1 * a3;
            const double r10 = s1 * a0 + c1 * a2, r11 = s1 * a1 + c1 * a3;
            A[p1 * ld + p2] = c2 * r00 - s2 * r01;
            A[p1 * ld + q2] = s2 * r00 + c2 * r01;
            A[q1 * ld + p2] = c2 * r10 - s2 * r11;
            A[q1 * ld + q2] = s2 * r10 + c2 * r11;
          } else {
            const int e2 = e - totA, i = e2 / half, R = e2 - (e2 / half) * half;
            const int p = pp[R], q = qq[R];
            const double c = cs[R], s = sn[R];
            const double v0 = V[i * ld + p], v1 = V[i * ld + q];
            V[i * ld + p] = c * v0 - s * v1;
            V[i * ld + q] = s * v0 + c * v1;
          }
        }
        __syncthreads();
        continue;
      }
      for (int base = 0; base < totA; base += CA * 256) {
        double a0[CA], a1[CA], a2[CA], a3[CA], c1v[CA], s1v[CA], c2v[CA], s2v[CA];
        int o0[CA], o1[CA], o2[CA], o3[CA];
        bool ok[CA];
#pragma unroll
        for (int j = 0; j < CA; ++j) {
          const int e = base + tid + j * 256;
          ok[j] = e < totA;
          // e = P * half + R (exact in float for e < 96 * 48)
          const int P = ok[j] ? (int)((float)e * inv_half + 0.5f * inv_half) : 0;
          const int R = ok[j] ? e - P * half : 0;
          const int p1 = pp[P], q1 = qq[P], p2 = pp[R], q2 = qq[R];
          c1v[j] = cs[P];
          s1v[j] = sn[P];
          c2v[j] = cs[R];
          s2v[j] = sn[R];
          o0[j] = p1 * ld + p2;
          o1[j] = p1 * ld + q2;
          o2[j] = q1 * ld + p2;
          o3[j] = q1 * ld + q2;
        }
#pragma unroll
        for (int j = 0; j < CA; ++j)
          if (ok[j]) {
            a0[j] = A[o0[j]];
            a1[j] = A[o1[j]];
            a2[j] = A[o2[j]];
            a3[j] = A[o3[j]];
          }
#pragma unroll
        for (int j = 0; j < CA; ++j)
          if (ok[j]) {
            const double c1 = c1v[j], s1 = s1v[j], c2 = c2v[j], s2 = s2v[j];
            const double r00 = c1 * a0[j] - s1 * a2[j], r01 = c1 * a1[j] - s1 * a3[j];
            const double r10 = s1 * a0[j] + c1 * a2[j], r11 = s1 * a1[j] + c1 * a3[j];
            A[o0[j]] = c2 * r00 - s2 * r01;
            A[o1[j]] = s2 * r00 + c2 * r01;
            A[o2[j]] = c2 * r10 - s2 * r11;
            A[o3[j]] = s2 * r10 + c2 * r11;
          }
      }
      for (int base = 0; base < totV; base += CV * 256) {
        double v0[CV], v1[CV], cv[CV], sv[CV];
        int ov0[CV], ov1[CV];
        bool ok[CV];
#pragma unroll
        for (int j = 0; j < CV; ++j) {
          const int e = base + tid + j * 256;
          ok[j] = e < totV;
          const int i = ok[j] ? (int)((float)e * inv_half + 0.5f * inv_half) : 0;
          const int R = ok[j] ? e - i * half : 0;
          cv[j] = cs[R];
          sv[j] = sn[R];
          ov0[j] = i * ld + pp[R];
          ov1[j] = i * ld + qq[R];
        }
#pragma unroll
        for (int j = 0; j < CV; ++j)
          if (ok[j]) {
            v0[j] = V[ov0[j]];
            v1[j] = V[ov1[j]];
          }
#pragma unroll
        for (int j = 0; j < CV; ++j)
          if (ok[j]) {
            V[ov0[j]] = cv[j] * v0[j] - sv[j] * v1[j];
            V[ov1[j]] = sv[j] * v0[j] + cv[j] * v1[j];
          }
      }
      __syncthreads();
    }
    if (!sweep_any) break;
  }

  // descending order by a parallel rank count (ties by index); the padding index of odd b is excluded
  for (int i = tid; i < b; i += blockDim.x) {
    const double di = A[i * ld + i];
    int rk = 0;
    for (int j = 0; j < b; ++j) {
      const double dj = A[j * ld + j];
      rk += (dj > di) || (dj == di && j < i);
    }
    rank_of[rk] = i;
  }
  __syncthreads();
  if (tid == 0) scal[slot] = (double)sweep;
  for (int c = tid; c < b; c += blockDim.x) eval[c] = A[rank_of[c] * ld + rank_of[c]];
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int i = e / b, c = e - (e / b) * b;
    evec[(int64_t)i * ldv + c] = V[i * ld + rank_of[c]];
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

// ------------------------------------------------------------------------------------------
// Bordering step of the inverse Cholesky factor of the stored basis's Gram, BF16 form.  With
// G_Q = Q^T Q = L L^T for the stored (rounded, not orthonormal) basis Q and Linv = L^{-1} lower
// triangular, appending w columns Q' gives the new block row [Linv21, Linv22] of Linv:
//   L21 = (Linv11 Q^T Q')^T, L22 = chol(Q'^T Q' - L21 L21^T), Linv22 = L22^{-1},
//   Linv21 = -Linv22 L21 Linv11.
// Workgroup 0 factors S = Q'^T Q' - L21 L21^T (w <= 64, symmetrised, in LDS), inverts L22 (one
// thread per column) and writes Linv22 into Linv and its transpose into LinvT; a pivot that is
// not positive sets scal[slot] = 1 (else 0).  The other workgroups clear the strips
// Linv[0:rq, rq:rq+w] and LinvT[rq:rq+w, 0:rq], which an earlier basis of other block widths may
// have written.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_border_chol(const double* __restrict__ Gq22, int ldg,
                                                     const double* __restrict__ P, int ldp, int w, int rq,
                                                     double* __restrict__ Linv, double* __restrict__ LinvT, int ld,
                                                     double* scal, int slot) {
  if (blockIdx.x > 0) {
    const int64_t total = (int64_t)rq * w;
    for (int64_t e = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)(gridDim.x - 1) * blockDim.x) {
      const int i = (int)(e / w), j = (int)(e % w);
      Linv[(int64_t)i * ld + rq + j] = 0.0;
      LinvT[(int64_t)(rq + j) * ld + i] = 0.0;
    }
    return;
  }
  __shared__ double A[64][65];
  __shared__ double B[64][65];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int i = e / w, j = e % w;
    double sij = 0.5 * (Gq22[(int64_t)i * ldg + j] + Gq22[(int64_t)j * ldg + i]);
    if (P) sij -= 0.5 * (P[(int64_t)i * ldp + j] + P[(int64_t)j * ldp + i]);
    A[i][j] = sij;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  // right-looking Cholesky, lower triangle: column c scaled by its pivot's root, then the
  // trailing lower triangle updated
  for (int c = 0; c < w; ++c) {
    const double d = A[c][c];
    if (!(d > 0.0)) {  // uniform: every thread read the same pivot
      if (tid == 0) bad = 1;
      break;
    }
    const double lc = sqrt(d);
    __syncthreads();  // every thread has read the pivot
    for (int i = c + tid; i < w; i += blockDim.x) A[i][c] = (i == c) ? lc : A[i][c] / lc;
    __syncthreads();
    const int n1 = w - c - 1;
    for (int e = tid; e < n1 * n1; e += blockDim.x) {
      const int i = c + 1 + e / n1, j = c + 1 + e % n1;
      if (j <= i) A[i][j] -= A[i][c] * A[j][c];
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) scal[slot] = (double)bad;
  if (bad) return;  // uniform
  // inverse of the lower-triangular factor, one column per thread: L x = e_j
  if (tid < w) {
    const int j = tid;
    for (int i = 0; i < w; ++i) {
      double x = 0.0;
      if (i == j) {
        x = 1.0 / A[j][j];
      } else if (i > j) {
        double sacc = 0.0;
        for (int l = j; l < i; ++l) sacc = fma(A[i][l], B[l][j], sacc);
        x = -sacc / A[i][i];
      }
      B[i][j] = x;
    }
  }
  __syncthreads();
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int i = e / w, j = e % w;
    const double v = B[i][j];
    Linv[(int64_t)(rq + i) * ld + rq + j] = v;
    LinvT[(int64_t)(rq + j) * ld + rq + i] = v;
  }
}

// scal[slot] = sum_i G[i][i] (fixed order: strided per-thread sums, then a tree)
__global__ __launch_bounds__(256) void k_trace(const double* __restrict__ G, int ld, int r, double* scal, int slot) {
  __shared__ double red[256];
  double sacc = 0.0;
  for (int i = threadIdx.x; i < r; i += 256) sacc += G[(int64_t)i * ld + i];
  red[threadIdx.x] = sacc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) scal[slot] = red[0];
}

}  // namespace

hipError_t launch_border_chol(hipStream_t s, const double* Gq22, int ldg, const double* P, int ldp, int w, int rq,
                              double* Linv, double* LinvT, int ld, double* scal, int slot) {
  if (w <= 0 || w > 64 || rq < 0) return hipErrorInvalidValue;
  const int64_t strip = (int64_t)rq * w;
  const unsigned extra = (unsigned)std::min<int64_t>(256, (strip + 255) / 256);
  hipLaunchKernelGGL(k_border_chol, dim3(1 + extra), dim3(256), 0, s, Gq22, ldg, P, ldp, w, rq, Linv, LinvT, ld, scal,
                     slot);
  return hipGetLastError();
}

hipError_t launch_trace(hipStream_t s, const double* G, int ld, int r, double* scal, int slot) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, G, ld, r, scal, slot);
  return hipGetLastError();
}

hipError_t launch_jacobi(hipStream_t s, const double* H, int ldh, int b, double* eval, double* evec, int ldv,
                         double* scal, int slot, int max_sweeps, int splits, int64_t sstride) {
  if (b <= 0 || b > kEigMax || splits <= 0) return hipErrorInvalidValue;
  const int bb = b + (b & 1);
  const size_t lds = (size_t)2 * bb * (bb + 1) * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((size_t)2 * kEigMax * (kEigMax + 1) * sizeof(double)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), lds, s, H, ldh, splits, sstride, b, eval, evec, ldv, scal, slot,
                     max_sweeps);
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
