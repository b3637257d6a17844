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
          const double x = fma(dd, dd, 4.0 * apq * apq);  // x > 0 here (|a_pq| above the tolerance)
          const double den = fabs(dd) + x * rsq_nr(x);
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
        // up to 32 columns: one pass over the 2 x 2 blocks of A and the row pairs of V, no chunking
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
    // as in k_jacobi_wave: stop when the next sweep would rotate nothing
    bool big = false;
    for (int e = tid; e < bb * bb; e += blockDim.x) {
      const int i = e / bb, j = e - (e / bb) * bb;
      big = big || (i < j && fabs(A[i * ld + j]) > tol);
    }
    if (!__syncthreads_or(big)) {
      ++sweep;
      break;
    }
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

// The same cyclic Jacobi for blocks of at most kJacWaveMax columns, in one wave.  At these sizes a
// round is a short chain of LDS round trips, and with four waves their barriers and the flag
// exchange took most of it.  Here the ballot of the rotating lanes decides a round directly, the
// pair indices are recomputed from the round number instead of read from a table, and each lane's
// blocks of A and row pairs of V (fixed for the whole solve) are gathered before any is updated,
// so a round costs one LDS trip for the rotation inputs and one for the operands.  The rotations,
// the tolerance and the output are those of k_jacobi.
constexpr int kJacWaveMax = 32;
// blocks up to this width go to the one-wave kernel: measured on warm starts, 32.2 against 41.4 us at 12
// columns and 43.6 against 60.4 at 16, but 150 against 119 at 24 and 272 against 170 at 32, where the
// lanes' four A blocks and eight V row pairs per round outweigh the barriers of four waves
constexpr int kJacWaveSmall = 16;

// Indices (p < q) of pair slot t in a round of the round-robin ordering over bb indices: slot 0
// keeps index 0, the other indices move one position per round.
__device__ inline void rr_pair(int t, int round, int bb, int& p, int& q) {
  const int nb1 = bb - 1;
  int x = t - 1 + round;
  x = (x >= nb1) ? x - nb1 : x;
  int y = bb - 2 - t + round;
  y = (y >= nb1) ? y - nb1 : y;
  const int pa = (t == 0) ? 0 : 1 + x;
  const int pb = 1 + y;
  p = min(pa, pb);
  q = max(pa, pb);
}

// Orders the LDS accesses of one wave around this point (a wave's LDS instructions execute in
// order; the wait and the clobber keep the compiler from moving loads or stores across it).
__device__ inline void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// x of lane l (wave-uniform l), as a scalar broadcast
__device__ inline double readlane_d(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// Cyclic Jacobi on the b x b symmetric A (LDS, row stride NB + 1, padded to even order bb with a zero
// row and column), accumulating the rotations into V (LDS, same layout, the identity on entry), by one
// whole wave with no barrier: the rotations, the tolerance test and the stopping rule of k_jacobi.  A
// round first loads every operand this lane updates (blocks (P, R) of A, e = P half + R, and row pairs
// (i, R) of V, e = i half + R; the indices come from the round number), then the rotating lanes
// compute their (c, s) from the pivots and publish them through cs / sn, and the update follows: the
// operand loads overlap the rotation arithmetic, which is the round's longest chain.  Slot counts are
// wave-uniform, so slots a small block does not need are skipped by scalar branches.  Returns the
// number of sweeps.
template <int NB>
__device__ int jacobi_wave_core(double* A, double* V, double* cs, double* sn, int b, double tol, int max_sweeps,
                                int lane) {
  constexpr int LD = NB + 1, NH = NB / 2;
  constexpr int NA = (NH * NH + kWave - 1) / kWave;  // blocks of A per lane
  constexpr int NV = (NB * NH + kWave - 1) / kWave;  // row pairs of V per lane
  const int bb = b + (b & 1), half = bb / 2, nb1 = bb - 1;
  const int totA = half * half, totV = bb * half;
  const int nA = (totA + kWave - 1) / kWave, nV = (totV + kWave - 1) / kWave;
  int aP[NA], aR[NA], vI[NV], vR[NV];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const int e = lane + j * kWave;
    aP[j] = (e < totA) ? e / half : -1;
    aR[j] = (e < totA) ? e - (e / half) * half : 0;
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int e = lane + j * kWave;
    vI[j] = (e < totV) ? e / half : -1;
    vR[j] = (e < totV) ? e - (e / half) * half : 0;
  }
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    bool sweep_any = false;
    for (int round = 0; round < nb1; ++round) {
      // operands of this lane's updates (unused slots read clamped, valid addresses)
      double a0[NA], a1[NA], a2[NA], a3[NA], v0[NV], v1[NV];
      int o0[NA], o1[NA], o2[NA], o3[NA], w0[NV], w1[NV];
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        if (j >= nA) break;
        int p1, q1, p2, q2;
        rr_pair(aP[j] < 0 ? 0 : aP[j], round, bb, p1, q1);
        rr_pair(aR[j], round, bb, p2, q2);
        o0[j] = p1 * LD + p2;
        o1[j] = p1 * LD + q2;
        o2[j] = q1 * LD + p2;
        o3[j] = q1 * LD + q2;
        a0[j] = A[o0[j]];
        a1[j] = A[o1[j]];
        a2[j] = A[o2[j]];
        a3[j] = A[o3[j]];
      }
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        if (j >= nV) break;
        int p, q;
        rr_pair(vR[j], round, bb, p, q);
        const int i = vI[j] < 0 ? 0 : vI[j];
        w0[j] = i * LD + p;
        w1[j] = i * LD + q;
        v0[j] = V[w0[j]];
        v1[j] = V[w1[j]];
      }
      bool mine = false;
      if (lane < half) {
        int p, q;
        rr_pair(lane, round, bb, p, q);
        const double apq = A[p * LD + q], app = A[p * LD + p], aqq = A[q * LD + q];
        // computed on every rotating lane and selected, so the three loads go out together.  The square
        // root is x rsq(x) with the refined reciprocal root (a few ulps, where the IEEE root is a longer
        // chain): the angle only needs to be close, the rotation is orthogonal through c = rsq(1 + t^2)
        const double dd = aqq - app;
        const double x = fma(dd, dd, 4.0 * apq * apq);
        const double den = fabs(dd) + x * rsq_nr(x);
        const double tt = (dd >= 0.0 ? 2.0 : -2.0) * apq * rcp_nr(den);
        const double cr = rsq_nr(fma(tt, tt, 1.0));
        mine = fabs(apq) > tol;
        cs[lane] = mine ? cr : 1.0;
        sn[lane] = mine ? tt * cr : 0.0;
      }
      if (__ballot(mine) == 0ull) continue;  // wave-uniform: nothing rotates this round
      sweep_any = true;
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        if (j >= nA) break;
        const int P = aP[j] < 0 ? 0 : aP[j], R = aR[j];
        const double c1 = cs[P], s1 = sn[P], c2 = cs[R], s2 = sn[R];
        if (aP[j] >= 0) {
          const double r00 = c1 * a0[j] - s1 * a2[j], r01 = c1 * a1[j] - s1 * a3[j];
          const double r10 = s1 * a0[j] + c1 * a2[j], r11 = s1 * a1[j] + c1 * a3[j];
          A[o0[j]] = c2 * r00 - s2 * r01;
          A[o1[j]] = s2 * r00 + c2 * r01;
          A[o2[j]] = c2 * r10 - s2 * r11;
          A[o3[j]] = s2 * r10 + c2 * r11;
        }
      }
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        if (j >= nV) break;
        const double c = cs[vR[j]], s = sn[vR[j]];
        if (vI[j] >= 0) {
          V[w0[j]] = c * v0[j] - s * v1[j];
          V[w1[j]] = s * v0[j] + c * v1[j];
        }
      }
      wave_lds_sync();
    }
    if (!sweep_any) break;
    // the sweep that would follow rotates nothing when every off-diagonal entry is at or below the
    // tolerance (no rotation changes A then): stop here with the count it would have ended with
    bool big = false;
    if (lane < bb)
      for (int i = 0; i < lane; ++i) big = big || fabs(A[i * LD + lane]) > tol;
    if (__ballot(big) == 0ull) {
      ++sweep;
      break;
    }
  }
  return sweep;
}

// The same cyclic Jacobi for blocks of at most kJacWaveMax columns, in one wave (jacobi_wave_core).
// At these sizes a round is a short chain of LDS round trips, and with four waves their barriers and
// the flag exchange took most of it.  The output is that of k_jacobi.
__global__ __launch_bounds__(kWave) void k_jacobi_wave(const double* __restrict__ H, int ldh, int splits,
                                                       int64_t sstride, int b, double* __restrict__ eval,
                                                       double* __restrict__ evec, int ldv, double* scal, int slot,
                                                       int max_sweeps) {
  constexpr int NB = kJacWaveMax, LD = NB + 1;
  __shared__ double A[NB * LD], V[NB * LD];
  __shared__ double cs[NB / 2], sn[NB / 2];
  __shared__ int rank_of[NB];
  const int lane = threadIdx.x;
  const int bb = b + (b & 1);
  for (int e = lane; e < bb * bb; e += kWave) {
    const int i = e / bb, j = e - (e / bb) * bb;
    double hij = 0.0, hji = 0.0;
    if (i < b && j < b) {
      hij = split_sum(H + (int64_t)i * ldh + j, splits, sstride);
      hji = split_sum(H + (int64_t)j * ldh + i, splits, sstride);
    }
    A[i * LD + j] = 0.5 * (hij + hji);
    V[i * LD + j] = (i == j) ? 1.0 : 0.0;
  }
  wave_lds_sync();
  double dm = 0.0;
  for (int i = lane; i < b; i += kWave) dm = fmax(dm, fabs(A[i * LD + i]));
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, kWave));
  const int sweep = jacobi_wave_core<NB>(A, V, cs, sn, b, 1e-15 * dm, max_sweeps, lane);
  wave_lds_sync();
  // descending order by a parallel rank count (ties by index); the padding index of odd b is excluded
  for (int i = lane; i < b; i += kWave) {
    const double di = A[i * LD + i];
    int rk = 0;
    for (int j = 0; j < b; ++j) {
      const double dj = A[j * LD + j];
      rk += (dj > di) || (dj == di && j < i);
    }
    rank_of[rk] = i;
  }
  wave_lds_sync();
  if (lane == 0) scal[slot] = (double)sweep;
  for (int c = lane; c < b; c += kWave) eval[c] = A[rank_of[c] * LD + rank_of[c]];
  for (int e = lane; e < b * b; e += kWave) {
    const int i = e / b, c = e - (e / b) * b;
    evec[(int64_t)i * ldv + c] = V[i * LD + rank_of[c]];
  }
}

// ------------------------------------------------------------------------------------------
// The subspace iteration of the block eigensolver for a small basis, one workgroup, nothing
// leaving LDS: G (r <= kSmallR) and the block (b <= kSmallB columns) are loaded once, then npairs
// double steps V <- CholeskyQR(p(G) V) (the last CholeskyQR twice), then the Rayleigh-Ritz step:
// H = V^T G V, its Jacobi eigenpairs (one wave, jacobi_wave_core), V <- V S, G V <- (G V) S and the
// residual norms.  p(G) V is alpha G (G V) + beta G V + V (the Chebyshev filter) or G (G V).  The
// products run on the FP64 matrix cores, one 16-row tile per wave; the CholeskyQR follows the rules
// of k_chol_trsm (a column whose pivot falls to dep_tol^2 of its Gram diagonal is dropped and the
// kept columns are packed to the left).  At these sizes every launch of the multi-kernel chain is a
// few microseconds of latency around a few hundred cycles of work; here the chain is one launch.
// Outputs: EV (Ritz vectors), GV (G times them), eval[0..b) (Ritz values, descending),
// eval[ldres + c] (residual norms), scal[slot] (Jacobi sweeps).
// ------------------------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));
__device__ inline dbl4 mfma16x16x4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kSmallThreads = 512;
constexpr int kSGL = kSmallR + 1;  // row stride of G in LDS (odd: the A operand's 16 rows fall on distinct banks)
constexpr int kJL = kSmallB + 1;   // row stride of the b x b blocks

// NB (8, 12 or 16, at least b) sizes the register arrays of the Cholesky factorisation and of the row
// solve; the LDS layout keeps 16 columns for the matrix-core tiles either way.
template <int NB>
__global__ __launch_bounds__(kSmallThreads) void k_eig_small(int r, const double* __restrict__ G, int ldg,
                                                             double* __restrict__ EV, double* __restrict__ GV, int ldv,
                                                             int b, int npairs, int filt, double alpha, double beta,
                                                             double dep_tol, double* __restrict__ eval, int ldres,
                                                             double* scal, int slot, int max_sweeps, int valid,
                                                             int ev_rows, uint64_t seed, uint64_t tag,
                                                             double* post_dst, unsigned* post_flag, unsigned post_seq) {
  __shared__ double Gs[kSmallR * kSGL];            // G; after the Rayleigh-Ritz products, (G V) S
  __shared__ double Vs[kSmallR * kSmallB];         // the block
  __shared__ double Ts[kSmallR * kSmallB];         // G V
  __shared__ double Zs[kSmallR * kSmallB];         // p(G) V; after the Rayleigh-Ritz products, V S
  __shared__ double Red[2 * 256];                  // the two waves' halves of a 16 x 16 product
  __shared__ double Cg[kSmallB * kJL];             // Gram, Cholesky factor, then the rows of R; later S
  __shared__ double JA[kSmallB * kJL], JV[kSmallB * kJL];
  __shared__ double cs[kSmallB / 2], sn[kSmallB / 2];
  __shared__ double rinv[kSmallB], theta[kSmallB], resid[2 * kSmallB];
  __shared__ int rank_of[kSmallB];
  __shared__ int keepm[1];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int RP = (r + 15) & ~15, RT = RP / 16;
  const int kl = lane >> 4, cl = lane & 15;

  // G in batches of eight loads per thread in flight (clamped, valid addresses; masked on store).  The
  // start block is drawn while the first batch is in flight: the kept columns (rows past ev_rows
  // zero) and Gaussian columns valid .. b-1, one Philox draw per row and group of four columns
  // (element (i, c) is z[c % 4] of the draw for (i, c / 4), as in k_fill_random).
  static_assert(kSmallR * (kSmallB / 4) <= kSmallThreads, "one group of four columns per thread");
  auto load_g = [&](int e0, double* gv) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + tid + u * kSmallThreads, i = e / RP, k = e - (e / RP) * RP;
      gv[u] = G[(int64_t)min(i, r - 1) * ldg + min(k, r - 1)];
    }
  };
  auto store_g = [&](int e0, const double* gv) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + tid + u * kSmallThreads, i = e / RP, k = e - (e / RP) * RP;
      if (e < RP * RP) Gs[i * kSGL + k] = (i < r && k < r) ? gv[u] : 0.0;
    }
  };
  {
    double gv[8];
    load_g(0, gv);
    if (tid < RP * (kSmallB / 4)) {
      const int i = tid / (kSmallB / 4), c0 = 4 * (tid % (kSmallB / 4));
      double z[4] = {0.0, 0.0, 0.0, 0.0};
      if (i < r && c0 + 3 >= valid && c0 < b)  // a Gaussian column in this group
        gaussian4((uint64_t)i, (uint64_t)(c0 / 4), tag, 0xFFFFFFFFull, seed, z);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u;
        double v = 0.0;
        if (i < r && c < valid)
          v = (i < ev_rows) ? EV[(int64_t)i * ldv + c] : 0.0;
        else if (i < r && c < b)
          v = z[u];
        Vs[i * kSmallB + c] = v;
      }
    }
    store_g(0, gv);
  }
  for (int e0 = 8 * kSmallThreads; e0 < RP * RP; e0 += 8 * kSmallThreads) {
    double gv[8];
    load_g(e0, gv);
    store_g(e0, gv);
  }
  __syncthreads();

  // Out = G In (RP x 16) on waves 0 .. RT - 1, then Out = alpha Out' + beta T + V when `mix`
  auto gprod = [&](const double* In, double* Out, bool mix) {
    if (wv < RT) {
      // four independent accumulator chains over interleaved k-steps, added in a fixed order
      dbl4 a4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] = dbl4{0.0, 0.0, 0.0, 0.0};
      const double* ga = Gs + (wv * 16 + cl) * kSGL;
      for (int k0 = 0; k0 < RP; k0 += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 4 * u + kl;
          a4[u] = mfma16x16x4(ga[k], In[k * kSmallB + cl], a4[u]);
        }
      }
      const dbl4 acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = (wv * 16 + kl + 4 * v) * kSmallB + cl;
        Out[o] = mix ? fma(alpha, acc[v], fma(beta, Ts[o], Vs[o])) : acc[v];
      }
    }
    __syncthreads();
  };
  // Red = X^T Y (16 x 16) over the RP rows, two waves taking half each; returns nothing (read Red)
  auto tprod = [&](const double* X, const double* Y) {
    if (wv < 2) {
      dbl4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
      const int h0 = wv * (RP / 2), h1 = h0 + RP / 2;  // RP / 2 is a multiple of 8
      for (int k0 = h0; k0 < h1; k0 += 8) {
        a0 = mfma16x16x4(X[(k0 + kl) * kSmallB + cl], Y[(k0 + kl) * kSmallB + cl], a0);
        a1 = mfma16x16x4(X[(k0 + 4 + kl) * kSmallB + cl], Y[(k0 + 4 + kl) * kSmallB + cl], a1);
      }
      const dbl4 acc = a0 + a1;
#pragma unroll
      for (int v = 0; v < 4; ++v) Red[wv * 256 + (kl + 4 * v) * 16 + cl] = acc[v];
    }
    __syncthreads();
  };
  // Vs <- Zs R^{-1}, Zs^T Zs = R^T R (CholeskyQR, the rules of k_chol_trsm)
  auto cholqr = [&]() {
    tprod(Zs, Zs);
    if (wv == 0) {
      // right-looking Cholesky in registers: lane i < NB holds row i of the symmetric Gram (both
      // triangles, updated alike, so it stays symmetric); step c reads the pivot and row c from lane c
      // (v_readlane, no LDS round trip) and lanes i > c subtract their multiple A[i][c] / A[c][c] of it
      // (the other lanes subtract zero).  Step c of a kept column leaves the pivot in piv on lane c.
      double a[NB];
      const int li = lane < NB ? lane : 0;
#pragma unroll
      for (int j = 0; j < NB; ++j) {  // a product with 0 or 1, not a select: the loads stay unconditional
        const double x = Red[li * 16 + j] + Red[256 + li * 16 + j];
        a[j] = x * ((lane < b && j < b) ? 1.0 : 0.0);
      }
      unsigned keep = 0;
      double gd[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        gd[c] = fmax(readlane_d(a[c], c), 0.0);
        if (c < b && gd[c] > 0.0) keep |= 1u << c;
      }
      double piv = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c >= b) break;  // uniform
        const double d = readlane_d(a[c], c);
        if (!((keep >> c & 1u) && d > dep_tol * dep_tol * gd[c] && d > 0.0)) {  // uniform
          keep &= ~(1u << c);
          continue;
        }
        piv = (lane == c) ? d : piv;
        const double f = (lane > c) ? a[c] * rcp_nr(d) : 0.0;
#pragma unroll
        for (int j = c + 1; j < NB; ++j) a[j] = fma(-f, readlane_d(a[j], c), a[j]);
      }
      // rows of R (row c on lane c): R[c][c] = sqrt(pivot), R[c][j] = A[c][j] / R[c][c]; zero rows and
      // columns for the dropped and inactive indices
      const bool kc = lane < b && (keep >> li & 1u);
      const double ri = kc ? rsq_nr(piv) : 0.0;
      if (lane < kSmallB) {
        rinv[lane] = ri;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          double v = 0.0;
          if (kc && j >= lane && (keep >> j & 1u)) v = a[j] * ri;  // j == lane: sqrt(pivot)
          Cg[lane * kJL + j] = v;
        }
      }
      if (lane == 0) keepm[0] = (int)keep;
    }
    __syncthreads();
    // forward substitution, one row per thread; kept columns packed to the left
    if (tid < RP) {
      double z[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) z[c] = Zs[tid * kSmallB + c];
      if constexpr (NB <= 8) {
        // every entry of R and every 1 / R[c][c] in registers first (all of them written, zeros past b),
        // so the substitution chain waits on no LDS load; past b it leaves the zero columns zero
        double rr[NB * (NB - 1) / 2 + 1], ri[NB];
        int t = 0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
#pragma unroll
          for (int l = 0; l < c; ++l) rr[t++] = Cg[l * kJL + c];
#pragma unroll
        for (int c = 0; c < NB; ++c) ri[c] = rinv[c];
        t = 0;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          double v = z[c];
#pragma unroll
          for (int l = 0; l < c; ++l) v = fma(-z[l], rr[t++], v);
          z[c] = v * ri[c];
        }
      } else {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          if (c < b) {
            double v = z[c];
#pragma unroll
            for (int l = 0; l < c; ++l) v = fma(-z[l], Cg[l * kJL + c], v);
            z[c] = v * rinv[c];
          }
        }
      }
      const unsigned keep = (unsigned)keepm[0];
      int q = 0;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < b && (keep >> c & 1u)) Vs[tid * kSmallB + q++] = (tid < r) ? z[c] : 0.0;
      for (int c = q; c < kSmallB; ++c) Vs[tid * kSmallB + c] = 0.0;
    }
    __syncthreads();
  };

  for (int pr = 0; pr < npairs; ++pr) {
    gprod(Vs, Ts, false);           // T = G V
    gprod(Ts, Zs, filt != 0);       // Z = alpha G T + beta T + V, or G T
    cholqr();
    if (pr + 1 == npairs) {         // the last pass before the Rayleigh-Ritz step runs twice
      for (int e = tid; e < RP * kSmallB; e += kSmallThreads) Zs[e] = Vs[e];
      __syncthreads();
      cholqr();
    }
  }

  // Rayleigh-Ritz: H = V^T G V (symmetrised), S Theta S^T = H
  gprod(Vs, Ts, false);
  tprod(Vs, Ts);
  if (wv == 0) {
    const int bb = b + (b & 1);
    for (int e = lane; e < kSmallB * kSmallB; e += kWave) {
      const int i = e >> 4, j = e & 15;
      double h = 0.0;
      if (i < b && j < b) h = 0.5 * ((Red[i * 16 + j] + Red[256 + i * 16 + j]) + (Red[j * 16 + i] + Red[256 + j * 16 + i]));
      if (i < bb && j < bb) {
        JA[i * kJL + j] = h;
        JV[i * kJL + j] = (i == j) ? 1.0 : 0.0;
      }
    }
    wave_lds_sync();
    double dm = 0.0;
    if (lane < b) dm = fabs(JA[lane * kJL + lane]);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, kWave));
    const int sweeps = jacobi_wave_core<kSmallB>(JA, JV, cs, sn, b, 1e-15 * dm, max_sweeps, lane);
    wave_lds_sync();
    if (lane < b) {
      const double di = JA[lane * kJL + lane];
      int rk = 0;
      for (int j = 0; j < b; ++j) {
        const double dj = JA[j * kJL + j];
        rk += (dj > di) || (dj == di && j < lane);
      }
      rank_of[rk] = lane;
    }
    wave_lds_sync();
    if (lane < b) theta[lane] = JA[rank_of[lane] * kJL + rank_of[lane]];
    for (int e = lane; e < kSmallB * kSmallB; e += kWave) {  // S (b x b, descending), zero elsewhere
      const int k = e >> 4, c = e & 15;
      Cg[k * kJL + c] = (k < b && c < b) ? JV[k * kJL + rank_of[c]] : 0.0;
    }
    if (lane == 0) scal[slot] = (double)sweeps;
  }
  __syncthreads();
  // V S -> Zs, (G V) S -> Gs (G is no longer needed)
  for (int e = tid; e < RP * kSmallB; e += kSmallThreads) {
    const int i = e / kSmallB, c = e % kSmallB;
    double zv = 0.0, zt = 0.0;
    for (int k = 0; k < b; ++k) {
      const double sk = Cg[k * kJL + c];
      zv = fma(Vs[i * kSmallB + k], sk, zv);
      zt = fma(Ts[i * kSmallB + k], sk, zt);
    }
    Zs[e] = zv;
    Gs[e] = zt;
  }
  __syncthreads();
  // residual norms || (G V S)_c - theta_c (V S)_c ||, wave w taking columns 2 w and 2 w + 1
  for (int c = 2 * wv; c < 2 * wv + 2 && c < b; ++c) {
    double acc = 0.0;
    for (int i = lane; i < r; i += kWave) {
      const double d = Gs[i * kSmallB + c] - theta[c] * Zs[i * kSmallB + c];
      acc = fma(d, d, acc);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (lane == 0) {
      eval[c] = theta[c];
      eval[ldres + c] = sqrt(acc);
      resid[c] = theta[c];
      resid[b + c] = sqrt(acc);
    }
  }
  for (int e = tid; e < r * kSmallB; e += kSmallThreads) {
    const int i = e / kSmallB, c = e % kSmallB;
    if (c < b) {
      EV[(int64_t)i * ldv + c] = Zs[e];
      GV[(int64_t)i * ldv + c] = Gs[e];
    }
  }
  // the Ritz values and residual norms to the host: the device copies above complete before the host
  // can act on them (it only enqueues work behind this kernel)
  if (post_dst != nullptr) {  // uniform
    __syncthreads();
    if (tid < 2 * b) post_dst[tid] = resid[tid];
    __threadfence_system();
    __syncthreads();
    if (tid == 0) {
      __threadfence_system();
      *(volatile unsigned*)post_flag = post_seq;
    }
  }
}

// P = alpha P + beta G + I (r x r, row stride ld): with P = G^2 on entry, the second-degree
// Chebyshev filter of the block eigensolver
__global__ __launch_bounds__(256) void k_cheb2(int r, double* __restrict__ P, const double* __restrict__ G, int ld,
                                               double alpha, double beta) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e / r), j = (int)(e - (e / r) * r);
  const int64_t o = (int64_t)i * ld + j;
  P[o] = fma(alpha, P[o], fma(beta, G[o], i == j ? 1.0 : 0.0));
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

// C[:, c] = S[:, c] (sigma_c - tau), D[:, c] = S[:, c] / sigma_c, sigma_c = sqrt(theta_c), c < k; zeros for
// k <= c < kpad.
__global__ void k_factor_coeffs(int r, int k, int kpad, const double* __restrict__ S, int lds_,
                                const double* __restrict__ theta, double tau, double* __restrict__ C,
                                double* __restrict__ D, int ldc, double* __restrict__ Sk) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)r * kpad) return;
  const int i = (int)(t / kpad), c = (int)(t % kpad);
  if (c >= k) {
    C[(int64_t)i * ldc + c] = 0.0;
    D[(int64_t)i * ldc + c] = 0.0;
    return;
  }
  const double sg = sqrt(theta[c]);
  const double v = S[(int64_t)i * lds_ + c];
  C[(int64_t)i * ldc + c] = v * (sg - tau);
  D[(int64_t)i * ldc + c] = v / sg;
  if (Sk) Sk[(int64_t)i * ldc + c] = v;  // the kept eigenvectors themselves, when asked for
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
  if (b <= kJacWaveSmall) {
    hipLaunchKernelGGL(k_jacobi_wave, dim3(1), dim3(kWave), 0, s, H, ldh, splits, sstride, b, eval, evec, ldv, scal,
                       slot, max_sweeps);
    return hipGetLastError();
  }
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

hipError_t launch_eig_small(hipStream_t s, int r, const double* G, int ldg, double* EV, double* GV, int ldv, int b,
                            int npairs, bool filt, double alpha, double beta, double dep_tol, double* eval, int ldres,
                            double* scal, int slot, int max_sweeps, int valid, int ev_rows, uint64_t seed,
                            uint64_t tag, double* post_dst, unsigned* post_flag, unsigned post_seq) {
  if (r <= 0 || r > kSmallR || b <= 0 || b > kSmallB || b > r || npairs < 1 || valid < 0 || valid > b) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b <= 8 ? k_eig_small<8> : b <= 12 ? k_eig_small<12> : k_eig_small<kSmallB>, dim3(1),
                     dim3(kSmallThreads), 0, s, r, G, ldg, EV,
                     GV, ldv, b, npairs, filt ? 1 : 0, alpha, beta, dep_tol, eval, ldres, scal, slot, max_sweeps, valid,
                     ev_rows, seed, tag, post_dst, post_flag, post_seq);
  return hipGetLastError();
}

hipError_t launch_cheb2(hipStream_t s, int r, double* P, const double* G, int ld, double alpha, double beta) {
  if (r <= 0) return hipSuccess;
  const int64_t n = (int64_t)r * r;
  hipLaunchKernelGGL(k_cheb2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r, P, G, ld, alpha, beta);
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
                                double tau, double* C, double* D, int ldc, double* Sk, int kpad) {
  kpad = std::max(kpad, k);
  if (kpad > ldc) return hipErrorInvalidValue;
  const int64_t work = (int64_t)r * kpad;
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL(k_factor_coeffs, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, r, k, kpad, S, lds_,
                     theta, tau, C, D, ldc, Sk);
  return hipGetLastError();
}

}  // namespace svt
