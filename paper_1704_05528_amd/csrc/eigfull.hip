// Full symmetric eigen-decomposition of the projected Gram G = W^T W (r x r, float64) for bases
// whose thresholded count does not fit the one-workgroup block solver of eig.hip.
//
// svd(B) of Alg. 3 needs every singular value of B above tau (Eq. 5); when that count k grows
// towards the basis width, subspace iteration on the leading block no longer pays, and the whole
// of G is diagonalised.  The adjoint of the thresholding map needs every eigenpair of G as well.
//
// Method: two-sided cyclic Jacobi (Golub & Van Loan, sym.schur2 rotations) in round-robin order,
// over many workgroups.  In one round the nn/2 disjoint index pairs (p, q) rotate at once: with
// J block diagonal over the pairs, row pair (p, q) of J^T A J depends only on rows p and q of A
// and on the rotations of all pairs.  The workgroup that owns a pair rewrites its two rows in
// place, so no workgroup reads another's rows within a round.  The only cross-workgroup data are
// the three entries (a_pp, a_qq, a_pq) each pair needs for its rotation: the owners of the rows
// write them for the next round's pairs into a small array (double buffered by round parity),
// and every workgroup of the next launch computes all rotations from it.  A round is one launch;
// kernel boundaries order the rounds.  The eigenvectors accumulate as the rows of Vt
// (V <- V J rotates rows p, q of V^T with the pair's own rotation).
#include "svt_internal.h"

#include <algorithm>

namespace svt {

namespace {

constexpr int kJgThreads = 256;

// Round-robin pairing of nn (even) indices: slot 0 keeps index 0, the other indices move by one
// position per round; every pair meets once in nn - 1 rounds.
__device__ inline void rr_pair(int t, int rd, int nn, int* p, int* q) {
  const int nb1 = nn - 1;
  int x = t - 1 + rd;
  x = (x >= nb1) ? x - nb1 : x;
  int y = nn - 2 - t + rd;
  y = (y >= nb1) ? y - nb1 : y;
  const int pa = (t == 0) ? 0 : 1 + x;
  const int pb = 1 + y;
  *p = min(pa, pb);
  *q = max(pa, pb);
}

// slot of index x in round rd, and its partner (inverse of rr_pair)
__device__ inline void rr_slot(int x, int rd, int nn, int* slot, int* partner) {
  const int nb1 = nn - 1;
  if (x == 0) {
    *slot = 0;
    int p, q;
    rr_pair(0, rd, nn, &p, &q);
    *partner = q;
    return;
  }
  // x = 1 + (t - 1 + rd) mod nb1 for a first position, x = 1 + (nn - 2 - t + rd) mod nb1 for a second
  int t1 = (x - 1 - rd) % nb1;
  t1 = (t1 < 0) ? t1 + nb1 : t1;
  t1 += 1;  // candidate slot as first position (slots 1 .. nb1)
  if (t1 <= nn / 2 - 1) {
    int p, q;
    rr_pair(t1, rd, nn, &p, &q);
    *slot = t1;
    *partner = (p == x) ? q : p;
    return;
  }
  int t2 = (nn - 2 + rd - (x - 1)) % nb1;
  t2 = (t2 < 0) ? t2 + nb1 : t2;
  int p, q;
  rr_pair(t2, rd, nn, &p, &q);
  *slot = t2;
  *partner = (p == x) ? q : p;
}

// rotation (c, s) annihilating a_pq, the smaller angle (as k_jacobi)
__device__ inline bool jg_rotation(double app, double aqq, double apq, double tol, double* c, double* s) {
  if (!(fabs(apq) > tol)) {
    *c = 1.0;
    *s = 0.0;
    return false;
  }
  const double dd = aqq - app;
  const double den = fabs(dd) + sqrt(fma(dd, dd, 4.0 * apq * apq));
  const double tt = (dd >= 0.0 ? 2.0 : -2.0) * apq / den;
  const double cc = 1.0 / sqrt(fma(tt, tt, 1.0));
  *c = cc;
  *s = tt * cc;
  return true;
}

__device__ inline double jg_wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// Replace A by its symmetric part, pad an odd order with a zero row and column (identity row of
// Vt) and set Vt = I when asked; grid-stride loops.
__global__ void k_jg_init(double* __restrict__ A, int lda, int n, int nn, double* __restrict__ Vt, int ldv,
                          int vt_identity, double* __restrict__ pin) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // symmetric part (a product like U^T G U is symmetric only up to rounding): each pair i < j once
  for (int64_t e = tid; e < (int64_t)n * n; e += stride) {
    const int64_t i = e / n, j = e - (e / n) * n;
    if (i < j) {
      const double v = 0.5 * (A[i * lda + j] + A[j * lda + i]);
      A[i * lda + j] = v;
      A[j * lda + i] = v;
    }
  }
  if (nn != n) {
    for (int64_t i = tid; i < nn; i += stride) {
      A[(int64_t)n * lda + i] = 0.0;
      A[i * lda + n] = 0.0;
    }
  }
  if (vt_identity) {
    for (int64_t e = tid; e < (int64_t)nn * nn; e += stride) {
      const int64_t i = e / nn, j = e - (e / nn) * nn;
      Vt[i * ldv + j] = (i == j) ? 1.0 : 0.0;
    }
  } else if (nn != n) {
    for (int64_t i = tid; i < nn; i += stride) {
      Vt[(int64_t)n * ldv + i] = (i == n) ? 1.0 : 0.0;
      Vt[i * ldv + n] = (i == n) ? 1.0 : 0.0;
    }
  }
}

// rotation inputs of round 0 and the threshold (1e-15 of the largest diagonal entry, as k_jacobi);
// one workgroup (the padding of an odd order is written by k_jg_init before)
__global__ __launch_bounds__(kJgThreads) void k_jg_start(const double* __restrict__ A, int lda, int n, int nn,
                                                         double* __restrict__ pin, double* __restrict__ tolp) {
  __shared__ double red[kJgThreads / kWave];
  const int tid = threadIdx.x;
  double dm = 0.0;
  for (int i = tid; i < n; i += kJgThreads) dm = fmax(dm, fabs(A[(int64_t)i * lda + i]));
  dm = jg_wave_max(dm);
  if ((tid & (kWave - 1)) == 0) red[tid / kWave] = dm;
  __syncthreads();
  if (tid == 0) {
    double t = red[0];
    for (int w = 1; w < kJgThreads / kWave; ++w) t = fmax(t, red[w]);
    *tolp = 1e-15 * t;
  }
  for (int t = tid; t < nn / 2; t += kJgThreads) {
    int p, q;
    rr_pair(t, 0, nn, &p, &q);
    pin[3 * t] = A[(int64_t)p * lda + p];
    pin[3 * t + 1] = A[(int64_t)q * lda + q];
    pin[3 * t + 2] = A[(int64_t)p * lda + q];
  }
}

// One round rd.  pin_cur: rotation inputs of this round (3 per slot); pin_next: those of round
// rd + 1 (mod nn - 1), written by the owners of the rows.  spw slots per workgroup.  flag is set
// to 1 when any pair rotates.
__global__ __launch_bounds__(kJgThreads) void k_jg_round(double* __restrict__ A, int lda, double* __restrict__ Vt,
                                                         int ldv, int nn, int rd, int spw,
                                                         const double* __restrict__ pin_cur,
                                                         double* __restrict__ pin_next, const double* __restrict__ tolp,
                                                         int32_t* __restrict__ flag) {
  extern __shared__ double jsm[];
  const int h = nn / 2;
  double* cs = jsm;
  double* sn = cs + h;
  int* pp = reinterpret_cast<int*>(sn + h);
  int* qq = pp + h;
  __shared__ int nslot[2 * 8], npart[2 * 8];  // next-round slot and partner of the owned rows (spw <= 8)
  const int tid = threadIdx.x;
  const double tol = *tolp;
  int any = 0;
  for (int t = tid; t < h; t += kJgThreads) {
    int p, q;
    rr_pair(t, rd, nn, &p, &q);
    double c, s;
    any |= jg_rotation(pin_cur[3 * t], pin_cur[3 * t + 1], pin_cur[3 * t + 2], tol, &c, &s) ? 1 : 0;
    cs[t] = c;
    sn[t] = s;
    pp[t] = p;
    qq[t] = q;
  }
  const int rdn = (rd + 1 == nn - 1) ? 0 : rd + 1;
  const int t0 = blockIdx.x * spw;
  const int nown = min(spw, h - t0);
  if (tid < 2 * nown) {
    const int t = t0 + tid / 2;
    int p, q;
    rr_pair(t, rd, nn, &p, &q);
    const int x = (tid & 1) ? q : p;
    int sl, pa;
    rr_slot(x, rdn, nn, &sl, &pa);
    nslot[tid] = sl;
    npart[tid] = pa;
  }
  any = __syncthreads_or(any);
  if (!any) {
    // nothing rotates: the rows are unchanged; pass on the next round's inputs
    if (tid < 2 * nown) {
      const int t = t0 + tid / 2;
      const int x = (tid & 1) ? qq[t] : pp[t];
      const int sl = nslot[tid], pa = npart[tid];
      const double* row = A + (int64_t)x * lda;
      if (x < pa) {
        pin_next[3 * sl] = row[x];
        pin_next[3 * sl + 2] = row[pa];
      } else {
        pin_next[3 * sl + 1] = row[x];
      }
    }
    return;
  }
  if (blockIdx.x == 0 && tid == 0) *flag = 1;
  for (int o = 0; o < nown; ++o) {
    const int P = t0 + o;
    const int p1 = pp[P], q1 = qq[P];
    const double c1 = cs[P], s1 = sn[P];
    double* rp = A + (int64_t)p1 * lda;
    double* rq = A + (int64_t)q1 * lda;
    const int nsp = nslot[2 * o], npp = npart[2 * o], nsq = nslot[2 * o + 1], npq = npart[2 * o + 1];
    // the 2 x 2 blocks (P, R) of the two rows, R over all slots: rows rotate with P's rotation,
    // columns with R's
    for (int R = tid; R < h; R += kJgThreads) {
      const int p2 = pp[R], q2 = qq[R];
      const double c2 = cs[R], s2 = sn[R];
      const double a0 = rp[p2], a1 = rp[q2], a2 = rq[p2], a3 = rq[q2];
      const double r00 = c1 * a0 - s1 * a2, r01 = c1 * a1 - s1 * a3;
      const double r10 = s1 * a0 + c1 * a2, r11 = s1 * a1 + c1 * a3;
      const double n00 = c2 * r00 - s2 * r01, n01 = s2 * r00 + c2 * r01;
      const double n10 = c2 * r10 - s2 * r11, n11 = s2 * r10 + c2 * r11;
      rp[p2] = n00;
      rp[q2] = n01;
      rq[p2] = n10;
      rq[q2] = n11;
      // inputs of the next round: the diagonal entries and the entry of each row at its next partner
      if (R == P) {
        if (p1 < npp) pin_next[3 * nsp] = n00; else pin_next[3 * nsp + 1] = n00;
        if (q1 < npq) pin_next[3 * nsq] = n11; else pin_next[3 * nsq + 1] = n11;
      }
      if (p1 < npp) {
        if (p2 == npp) pin_next[3 * nsp + 2] = n00;
        if (q2 == npp) pin_next[3 * nsp + 2] = n01;
      }
      if (q1 < npq) {
        if (p2 == npq) pin_next[3 * nsq + 2] = n10;
        if (q2 == npq) pin_next[3 * nsq + 2] = n11;
      }
    }
    if (s1 != 0.0) {
      double* vp = Vt + (int64_t)p1 * ldv;
      double* vq = Vt + (int64_t)q1 * ldv;
      for (int i = tid; i < nn; i += kJgThreads) {
        const double x = vp[i], y = vq[i];
        vp[i] = c1 * x - s1 * y;
        vq[i] = s1 * x + c1 * y;
      }
    }
  }
}

// part[b] = max |A_ij|, j > i, over this workgroup's rows (grid-stride over rows).  The rotations
// read the upper triangle (a_pq with p < q), so its maximum decides whether a sweep would rotate.
__global__ __launch_bounds__(kJgThreads) void k_jg_offmax(const double* __restrict__ A, int lda, int nn,
                                                          double* __restrict__ part) {
  __shared__ double red[kJgThreads / kWave];
  double v = 0.0;
  for (int i = blockIdx.x; i < nn; i += gridDim.x) {
    const double* row = A + (int64_t)i * lda;
    for (int j = i + 1 + threadIdx.x; j < nn; j += kJgThreads) v = fmax(v, fabs(row[j]));
  }
  v = jg_wave_max(v);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < kJgThreads / kWave; ++w) t = fmax(t, red[w]);
    part[blockIdx.x] = t;
  }
}

// out[0] = max over nb partial maxima, out[1] = the threshold
__global__ __launch_bounds__(kJgThreads) void k_jg_offmax_finish(const double* __restrict__ part, int nb,
                                                                 const double* __restrict__ tolp,
                                                                 double* __restrict__ out) {
  __shared__ double red[kJgThreads / kWave];
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += kJgThreads) v = fmax(v, part[b]);
  v = jg_wave_max(v);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < kJgThreads / kWave; ++w) t = fmax(t, red[w]);
    out[0] = t;
    out[1] = *tolp;
  }
}

// perm[rank] = i, ranks by descending diagonal (ties by index), eval[rank] = A_ii, for i < n
__global__ void k_jg_rank(const double* __restrict__ A, int lda, int n, int32_t* __restrict__ perm,
                          double* __restrict__ eval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = A[(int64_t)i * lda + i];
  int rk = 0;
  for (int j = 0; j < n; ++j) {
    const double dj = A[(int64_t)j * lda + j];
    rk += (dj > di) || (dj == di && j < i);
  }
  perm[rk] = i;
  eval[rk] = di;
}

// Et[c][l] = Vt[perm[c]][l] and EU[l][c] = Vt[perm[c]][l] for c, l < n (either output may be NULL)
__global__ void k_jg_gather(const double* __restrict__ Vt, int ldv, int n, const int32_t* __restrict__ perm,
                            double* __restrict__ Et, int ldet, double* __restrict__ EU, int ldeu) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int c = (int)(e / n), l = (int)(e - (e / n) * n);
  const double v = Vt[(int64_t)perm[c] * ldv + l];
  if (Et) Et[(int64_t)c * ldet + l] = v;
  if (EU) EU[(int64_t)l * ldeu + c] = v;
}

// Extend an orthogonal r0 x r0 matrix to r x r by the identity on the new rows and columns.
__global__ void k_extend_identity(double* __restrict__ M, int ld, int r0, int r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e / r), j = (int)(e - (e / r) * r);
  if (i < r0 && j < r0) return;
  M[(int64_t)i * ld + j] = (i == j) ? 1.0 : 0.0;
}

// dst[j][i] = src[i][j] for i < rows, j < cols (32 x 32 tiles through LDS)
__global__ void k_transpose(const double* __restrict__ src, int lds_, int rows, int cols, double* __restrict__ dst,
                            int ldd) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows per pass
  for (int yy = ty; yy < 32; yy += 8) {
    const int i = by + yy, j = bx + tx;
    if (i < rows && j < cols) tile[yy][tx] = src[(int64_t)i * lds_ + j];
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int j = bx + yy, i = by + tx;
    if (i < rows && j < cols) dst[(int64_t)j * ldd + i] = tile[tx][yy];
  }
}

inline unsigned jg_blocks(int64_t work, int per = 256) { return (unsigned)std::max<int64_t>(1, (work + per - 1) / per); }

}  // namespace

int jg_slots_per_wg(int nn) { return std::max(1, (nn / 2 + kJgMaxWg - 1) / kJgMaxWg); }

hipError_t launch_jg_start(hipStream_t s, double* A, int lda, int n, double* Vt, int ldv, bool vt_identity,
                           double* pin, double* tolp) {
  if (n <= 0 || n > kJgMaxOrder) return hipErrorInvalidValue;
  const int nn = n + (n & 1);
  hipLaunchKernelGGL(k_jg_init, dim3(jg_blocks((int64_t)nn * nn, 256 * 16)), dim3(256), 0, s, A, lda, n, nn, Vt, ldv,
                     vt_identity ? 1 : 0, pin);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_jg_start, dim3(1), dim3(kJgThreads), 0, s, A, lda, n, nn, pin, tolp);
  return hipGetLastError();
}

hipError_t launch_jg_round(hipStream_t s, double* A, int lda, double* Vt, int ldv, int nn, int rd, const double* pin_cur,
                           double* pin_next, const double* tolp, int32_t* flag) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jg_round, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((size_t)kJgMaxOrder / 2 * (2 * sizeof(double) + 2 * sizeof(int))));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (nn <= 0 || (nn & 1) || nn > kJgMaxOrder + 1 || rd < 0 || rd >= nn - 1) return hipErrorInvalidValue;
  const int spw = jg_slots_per_wg(nn);
  if (spw > 8) return hipErrorInvalidValue;
  const int h = nn / 2;
  const unsigned g = (unsigned)((h + spw - 1) / spw);
  const size_t lds = (size_t)h * (2 * sizeof(double) + 2 * sizeof(int));
  hipLaunchKernelGGL(k_jg_round, dim3(g), dim3(kJgThreads), lds, s, A, lda, Vt, ldv, nn, rd, spw, pin_cur, pin_next,
                     tolp, flag);
  return hipGetLastError();
}

hipError_t launch_jg_offmax(hipStream_t s, const double* A, int lda, int nn, const double* tolp, double* part,
                            double* out) {
  const int nb = std::min(nn, 256);
  hipLaunchKernelGGL(k_jg_offmax, dim3(nb), dim3(kJgThreads), 0, s, A, lda, nn, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_jg_offmax_finish, dim3(1), dim3(kJgThreads), 0, s, part, nb, tolp, out);
  return hipGetLastError();
}

hipError_t launch_jg_finish(hipStream_t s, const double* A, int lda, const double* Vt, int ldv, int n, int32_t* perm,
                            double* eval, double* Et, int ldet, double* EU, int ldeu) {
  hipLaunchKernelGGL(k_jg_rank, dim3(jg_blocks(n)), dim3(256), 0, s, A, lda, n, perm, eval);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_jg_gather, dim3(jg_blocks((int64_t)n * n)), dim3(256), 0, s, Vt, ldv, n, perm, Et, ldet, EU,
                     ldeu);
  return hipGetLastError();
}

hipError_t launch_extend_identity(hipStream_t s, double* M, int ld, int r0, int r) {
  if (r <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_extend_identity, dim3(jg_blocks((int64_t)r * r)), dim3(256), 0, s, M, ld, r0, r);
  return hipGetLastError();
}

hipError_t launch_transpose(hipStream_t s, const double* src, int lds_, int rows, int cols, double* dst, int ldd) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32)), dim3(256), 0, s,
                     src, lds_, rows, cols, dst, ldd);
  return hipGetLastError();
}

}  // namespace svt
