// Streaming kernels of the SVT / R4SVD hot path for gfx950 (wave64).
//
// Kernels that touch the iterate Y, the basis Q, the projection W = Y^T Q, sampled blocks
// and the factors of X are templates over the storage type T: double in the FP64 form,
// float in the mixed form.  Sparse products and the sampled product accumulate in T; Gram
// matrices, norms and every reduction accumulate in double.
//
// Every reduction is deterministic: per-workgroup partial sums in a fixed butterfly order,
// then one workgroup adds the partials in index order.  No floating-point atomics are used.
#include "svt_internal.h"

#include <type_traits>

#include <algorithm>

namespace svt {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over the workgroup; the result is valid in thread 0.
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

// om[j, c] for rows j < n and block columns c0 <= c < c0 + w (c0 a multiple of 4), stored at om[j*ld + c - c0].
template <class T>
__global__ void k_omega(T* __restrict__ om, int n, int c0, int w, int ld, uint64_t seed, uint64_t blk, uint64_t it) {
  const int ng = (w + 3) / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * ng) return;
  const int j = (int)(t / ng), g = (int)(t % ng);
  double z[4];
  gaussian4((uint64_t)j, (uint64_t)(c0 / 4 + g), blk, it, seed, z);
#pragma unroll
  for (int l = 0; l < 4; ++l)
    if (4 * g + l < w) om[(int64_t)j * ld + 4 * g + l] = (T)z[l];
}

// Gaussian fill of columns [c0, c1) of a rows x ld block (eigensolver start vectors): element (i, c)
// is z[c % 4] of the Philox draw for row i and column group c / 4.
__global__ void k_fill_random(double* __restrict__ V, int rows, int ld, int c0, int c1, uint64_t seed, uint64_t tag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = c1 - c0;
  if (t >= (int64_t)rows * w) return;
  const int i = (int)(t / w), c = c0 + (int)(t % w);
  double z[4];
  gaussian4((uint64_t)i, (uint64_t)(c / 4), tag, 0xFFFFFFFFull, seed, z);
  V[(int64_t)i * ld + c] = z[c % 4];
}

// columns c0 .. c0+count-1 of a rows x ld block set to the unit vectors e_{row0}, e_{row0+1}, ...
__global__ void k_set_unit(double* __restrict__ V, int rows, int ld, int c0, int count, int row0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * count) return;
  const int i = (int)(t / count), q = (int)(t % count);
  V[(int64_t)i * ld + c0 + q] = (i == row0 + q) ? 1.0 : 0.0;
}

// ------------------------------------------------------------------------------------------
// Segment-gather SpMM: out[row, :] = sum_{p in seg(row)} val[vperm(p)] * D[idx[p], :].
// With CSC segments (idx = row indices, D = Q) this is W = Y^T Q; with CSR segments
// (idx = column indices, vperm = CSR->CSC map, D = Omega) it is X = Y Omega.
// ------------------------------------------------------------------------------------------

// Four consecutive entries of a row of D (float, double or bfloat16) as T, entries from `valid`
// on as zero.  With vec (the four are in range and 16-byte aligned for float and double, 8-byte
// aligned for bfloat16) they come as one or two vector loads.
template <class T, class TD>
__device__ inline void load_row4(const TD* src, bool vec, int valid, T (&d)[4]) {
  if constexpr (std::is_same<TD, float>::value) {
    if (vec) {
      typedef float f4 __attribute__((ext_vector_type(4)));
      const f4 x = *reinterpret_cast<const f4*>(src);
      d[0] = x.x;
      d[1] = x.y;
      d[2] = x.z;
      d[3] = x.w;
      return;
    }
  } else if constexpr (std::is_same<TD, double>::value) {
    if (vec) {
      typedef double d2 __attribute__((ext_vector_type(2)));
      const d2 v0 = reinterpret_cast<const d2*>(src)[0], v1 = reinterpret_cast<const d2*>(src)[1];
      d[0] = v0.x;
      d[1] = v0.y;
      d[2] = v1.x;
      d[3] = v1.y;
      return;
    }
  } else {
    static_assert(std::is_same<TD, bf16>::value, "float, double or bf16 rows");
    if (vec) {
      const uint2 x = *reinterpret_cast<const uint2*>(src);  // entries 0, 1 in x.x (low half first)
      d[0] = (T)__builtin_bit_cast(float, x.x << 16);
      d[1] = (T)__builtin_bit_cast(float, x.x & 0xffff0000u);
      d[2] = (T)__builtin_bit_cast(float, x.y << 16);
      d[3] = (T)__builtin_bit_cast(float, x.y & 0xffff0000u);
      return;
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) d[c] = (c < valid) ? (T)src[c] : (T)0;
}

// rows of D may be loaded four entries at a time: 16-byte (float, double) or 8-byte (bf16) alignment
template <class TD>
inline bool rows_vec4(const TD* D, int ldd) {
  const uintptr_t align = sizeof(TD) == 2 ? 7u : 15u;
  return (ldd % 4 == 0) && ((reinterpret_cast<uintptr_t>(D) & align) == 0);
}

// Narrow blocks (w <= 16): a segment is shared by SPLIT waves (1: one segment per wave; 4: one
// per workgroup, for long segments); their lanes form 16 SPLIT groups of four, group gg takes the
// nonzeros p0 + gg, p0 + gg + 16 SPLIT, ..., and lane q of a group the columns 4q .. 4q + 3 of D's
// row (one 16-byte load for float when the row is aligned).  Each lane keeps four partial sums;
// a wave adds its 16 groups with four butterfly steps, and the SPLIT waves' sums are added in
// wave order (fixed order, deterministic).
template <int WN, int SPLIT, class T, class TD>
__global__ __launch_bounds__(256) void k_seg_spmm_narrow(int nrows, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx,
                                                         const int32_t* __restrict__ vperm, const T* __restrict__ val,
                                                         const TD* __restrict__ D, int ldd, T* __restrict__ out,
                                                         int ldo, int w, const int32_t* __restrict__ seg_lo,
                                                         const int32_t* __restrict__ seg_hi,
                                                         const int32_t* __restrict__ skip) {
  static_assert(WN == 16, "four lanes of four columns");
  static_assert(SPLIT == 1 || SPLIT == 4, "one segment per wave or per workgroup");
  constexpr int kU = 4;  // nonzeros per lane in flight
  constexpr int kG = 16 * SPLIT;  // lane groups per segment
  __shared__ T red[SPLIT][WN];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int row = blockIdx.x * (4 / SPLIT) + wave / SPLIT, sub = wave % SPLIT;
  if (row >= nrows) return;                         // uniform over the waves of a segment
  if (skip != nullptr && skip[row] != 0) return;  // uniform over the waves of a segment
  const int gg = sub * 16 + (lane >> 2), c0 = (lane & 3) * 4;
  const uintptr_t align = sizeof(TD) == 2 ? 7u : 15u;
  const bool vec = (sizeof(T) == 4 || sizeof(TD) == 2) && (c0 + 4 <= w) && (ldd % 4 == 0) &&
                   ((reinterpret_cast<uintptr_t>(D) & align) == 0);
  T acc[4] = {(T)0, (T)0, (T)0, (T)0};
  const int p0 = seg_lo ? seg_lo[row] : ptr[row], p1 = seg_lo ? seg_hi[row] : ptr[row + 1];
  for (int base = p0 + gg; base < p1; base += kG * kU) {
    T v[kU], d[kU][4];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int p = base + kG * u;
      const bool ok = p < p1;
      const int pc = ok ? p : p0;  // a valid position (the segment is not empty here)
      v[u] = ok ? val[vperm ? vperm[pc] : pc] : (T)0;
      load_row4<T, TD>(D + (int64_t)idx[pc] * ldd + c0, vec, w - c0, d[u]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = fma(v[u], d[u][c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int o = 4; o < kWave; o <<= 1) acc[c] += __shfl_xor(acc[c], o, kWave);
  }
  if constexpr (SPLIT > 1) {
    if (lane < 4) {
#pragma unroll
      for (int c = 0; c < 4; ++c) red[sub][c0 + c] = acc[c];
    }
    __syncthreads();
    if (sub != 0 || lane >= 4) return;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T t = red[0][c0 + c];
#pragma unroll
      for (int q = 1; q < SPLIT; ++q) t += red[q][c0 + c];
      acc[c] = t;
    }
  }
  if (lane < 4) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c0 + c < w) out[(int64_t)row * ldo + c0 + c] = acc[c];
  }
}

// Wide blocks: lanes over output columns (CPL = 4 per lane), nonzeros broadcast across the wave.
// Four nonzeros' rows of D are loaded before their products issue; with VEC the four columns of a
// lane come as one 16-byte (float) or two 16-byte (double) loads (ldd % 4 == 0, D 16-byte aligned).
// Segment forms: with seg_lo / seg_hi, "row" s is the position range [seg_lo[s], seg_hi[s]) and
// writes out row s (the chunk partials of long segments); with skip, rows whose flag is set are
// left to that chunked form.
template <int CPL, bool VEC, class T, class TD>
__global__ __launch_bounds__(256) void k_seg_spmm_wide(int nrows, const int32_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ idx,
                                                       const int32_t* __restrict__ vperm, const T* __restrict__ val,
                                                       const TD* __restrict__ D, int ldd, T* __restrict__ out, int ldo,
                                                       int w, const int32_t* __restrict__ seg_lo,
                                                       const int32_t* __restrict__ seg_hi,
                                                       const int32_t* __restrict__ skip) {
  static_assert(CPL == 4, "four columns per lane");
  const int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= nrows) return;
  if (skip != nullptr && skip[row] != 0) return;
  const int c0 = blockIdx.y * (kWave * CPL) + lane * CPL;
  const bool vec = VEC && (c0 + CPL <= w);
  T acc[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = (T)0;
  auto load4 = [&](int ii, T (&d)[CPL]) { load_row4<T, TD>(D + (int64_t)ii * ldd + c0, vec, w - c0, d); };
  const int p0 = seg_lo ? seg_lo[row] : ptr[row], p1 = seg_lo ? seg_hi[row] : ptr[row + 1];
  for (int base = p0; base < p1; base += kWave) {
    const int p = base + lane;
    int my_i = 0;
    T my_v = (T)0;
    if (p < p1) {
      my_i = idx[p];
      my_v = val[vperm ? vperm[p] : p];
    }
    const int cnt = min(kWave, p1 - base);
    int t = 0;
    for (; t + 4 <= cnt; t += 4) {
      T d0[CPL], d1[CPL], d2[CPL], d3[CPL];
      const int i0 = __shfl(my_i, t, kWave), i1 = __shfl(my_i, t + 1, kWave);
      const int i2 = __shfl(my_i, t + 2, kWave), i3 = __shfl(my_i, t + 3, kWave);
      load4(i0, d0);
      load4(i1, d1);
      load4(i2, d2);
      load4(i3, d3);
      const T v0 = __shfl(my_v, t, kWave), v1 = __shfl(my_v, t + 1, kWave);
      const T v2 = __shfl(my_v, t + 2, kWave), v3 = __shfl(my_v, t + 3, kWave);
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        acc[c] = fma(v0, d0[c], acc[c]);
        acc[c] = fma(v1, d1[c], acc[c]);
        acc[c] = fma(v2, d2[c], acc[c]);
        acc[c] = fma(v3, d3[c], acc[c]);
      }
    }
    for (; t < cnt; ++t) {
      T d0[CPL];
      load4(__shfl(my_i, t, kWave), d0);
      const T v0 = __shfl(my_v, t, kWave);
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[c] = fma(v0, d0[c], acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c)
    if (c0 + c < w) out[(int64_t)row * ldo + c0 + c] = acc[c];
}

// out[lcol[t], c] = sum of the chunk partials P[q, c], q = lfirst[t] .. lfirst[t+1]-1, for the long
// segments t (fixed order)
template <class T>
__global__ __launch_bounds__(256) void k_seg_chunk_sum(const int32_t* __restrict__ lcol,
                                                       const int32_t* __restrict__ lfirst, const T* __restrict__ P,
                                                       int ldp, T* __restrict__ out, int ldo, int w) {
  const int t = blockIdx.y, c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= w) return;
  const int q0 = lfirst[t];
  out[(int64_t)lcol[t] * ldo + c] = split_sum<T>(P + (int64_t)q0 * ldp + c, lfirst[t + 1] - q0, ldp);
}

// ------------------------------------------------------------------------------------------
// LDS-tiled W = Y^T Q for inputs where most RT x JB tiles of Y hold observed entries (image-
// like sampling densities).  A workgroup owns JB columns of Y (rows of W) and CB columns of Q;
// for each RT-row tile it scatters the tile's observed values into a zero-filled LDS tile,
// stages Q[i0:i0+RT, c0:c0+CB], and accumulates 4 x 4 register blocks.  tstart[j*(nt+1)+t] is
// the first CSC position of column j with row >= t*RT (built once from the fixed pattern).
// Row tiles are split over blockIdx.z; split s writes its sum to out + s * split_stride.
// ------------------------------------------------------------------------------------------
constexpr int kTR = 32, kTJ = 64, kTC = 64;

template <class T, class TQ>
__global__ __launch_bounds__(256) void k_spmm_t_tiled(int m, int n, const int32_t* __restrict__ rowidx,
                                                      const int32_t* __restrict__ tstart, int nt,
                                                      const T* __restrict__ val, const TQ* __restrict__ Q, int ldq,
                                                      int r, T* __restrict__ out, int ldo, int tiles_per_split,
                                                      int64_t split_stride) {
  __shared__ T Ys[kTR][kTJ + 2];
  __shared__ T Qs[kTR][kTC + 2];
  const int tid = threadIdx.x;
  const int j0 = blockIdx.x * kTJ, c0 = blockIdx.y * kTC;
  const int tj = tid / 16, tc = tid % 16;
  const int t_begin = blockIdx.z * tiles_per_split, t_end = min(nt, t_begin + tiles_per_split);
  T acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = (T)0;
  // scatter roles: 4 threads per column j of the tile
  const int sj = tid / 4, ssub = tid % 4;
  const int gj = j0 + sj;
  for (int t = t_begin; t < t_end; ++t) {
    const int i0 = t * kTR;
    for (int e = tid; e < kTR * kTJ; e += 256) Ys[e / kTJ][e % kTJ] = (T)0;
    for (int e = tid; e < kTR * kTC; e += 256) {
      const int i = e / kTC, c = e % kTC;
      Qs[i][c] = (i0 + i < m && c0 + c < r) ? (T)Q[(int64_t)(i0 + i) * ldq + c0 + c] : (T)0;
    }
    __syncthreads();
    if (gj < n) {
      const int p1 = tstart[(int64_t)gj * (nt + 1) + t + 1];
      for (int p = tstart[(int64_t)gj * (nt + 1) + t] + ssub; p < p1; p += 4) Ys[rowidx[p] - i0][sj] = val[p];
    }
    __syncthreads();
#pragma unroll 8
    for (int i = 0; i < kTR; ++i) {
      T a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = Ys[i][tj * 4 + u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = Qs[i][tc * 4 + v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
  T* o = out + blockIdx.z * split_stride;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + tj * 4 + u;
    if (j >= n) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = c0 + tc * 4 + v;
      if (c < r) o[(int64_t)j * ldo + c] = acc[u][v];
    }
  }
}

// W[j, c] = sum_s partial[s][j][c] (fixed order)
template <class T>
__global__ void k_split_sum(int n, int r, const T* __restrict__ partial, int splits, int64_t split_stride, int ldp,
                            T* __restrict__ W, int ldw) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * r) return;
  const int j = (int)(t / r), c = (int)(t % r);
  W[(int64_t)j * ldw + c] = split_sum<T>(partial + (int64_t)j * ldp + c, splits, split_stride);
}

// ------------------------------------------------------------------------------------------
// FP64 matrix cores.  v_mfma_f64_16x16x4f64 (one wave) takes the A operand (16 x 4) as
// A[l % 16][l / 16] in lane l, the B operand (4 x 16) as B[l / 16][l % 16], and accumulates the
// 16 x 16 result with rows (l / 16) + 4 v, v = 0..3, of column l % 16 in lane l.  Operands of
// float storage are widened to double on load.
// ------------------------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kUnroll = 8;  // k-steps whose operands are loaded before their products issue

__device__ inline dbl4 mfma_f64_16x16x4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Sum the accumulators of the NW waves of a workgroup in wave order (deterministic); the result
// is valid in wave 0.
template <int NW = 4>
__device__ inline dbl4 reduce_waves(dbl4 acc, double (*red)[kWave][4]) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  if (wv > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wv - 1][lane][v] = acc[v];
  }
  __syncthreads();
  if (wv == 0) {
    // wave order; one 4-double row of partner g per step keeps few values live
#pragma unroll 4
    for (int g = 0; g < NW - 1; ++g) {
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] += red[g][lane][v];
    }
  }
  return acc;
}

// ------------------------------------------------------------------------------------------
// The same product for tall operands with many tiles (the factor products of a large problem): a
// workgroup of four waves takes 64 rows x 32 columns, wave v the rows 16 v .. 16 v + 15 over the
// whole K range (no reduction) and both 16-column tiles, which share its loads of A; the four waves
// read the same slices of M at about the same time, mostly from L1.  One 16 x 16 tile per workgroup
// re-read its slice of M per 16 rows and the rows of A per 16 columns (about 50 GB from L2 for the
// factors of a 150000-row problem at r = 4096, k = 105).  No Gram epilogue.
// ------------------------------------------------------------------------------------------
constexpr int kTallRows = 64, kTallCols = 32;

template <class TA, class TM, class TO>
__global__ __launch_bounds__(4 * kWave) void k_rowmul_tall(RowmulProblem<TA, TM, TO> pr0,
                                                          RowmulProblem<TA, TM, TO> pr1) {
  const RowmulProblem<TA, TM, TO>& pr = blockIdx.z == 0 ? pr0 : pr1;
  const int rows = pr.rows, K = pr.K, lda = pr.lda, ldm = pr.ldm, ldo = pr.ldo, w = pr.w;
  const TA* __restrict__ A = pr.A;
  const TM* __restrict__ M = pr.M;
  TO* __restrict__ out = pr.out;
  const double alpha = pr.alpha, beta = pr.beta;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int i0 = blockIdx.x * kTallRows + 16 * wv, j0 = blockIdx.y * kTallCols;
  if (i0 >= rows || j0 >= w) return;  // uniform over the wave; the waves share no barrier
  const int ia = i0 + (lane & 15), jb0 = j0 + (lane & 15), jb1 = jb0 + 16, kl = lane >> 4;
  const bool rowok = ia < rows, c0ok = jb0 < w, c1ok = jb1 < w;
  // out-of-range operands are loaded from a clamped, valid address and replaced by zero
  const TA* arow = A + (int64_t)min(ia, rows - 1) * lda;
  const TM* mc0 = M + min(jb0, w - 1);
  const TM* mc1 = M + min(jb1, w - 1);
  const int steps = (K + 3) / 4;
  dbl4 a00 = {0.0, 0.0, 0.0, 0.0}, a01 = a00, a10 = a00, a11 = a00;
  for (int st = 0; st < steps; st += kUnroll) {
    TA ar[kUnroll];
    TM b0[kUnroll], b1[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int kc = min((st + u) * 4 + kl, K - 1);
      ar[u] = arow[kc];
      b0[u] = mc0[(int64_t)kc * ldm];
      b1[u] = mc1[(int64_t)kc * ldm];
    }
    double a[kUnroll], x0[kUnroll], x1[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const bool ok = (st + u < steps) && ((st + u) * 4 + kl < K);
      a[u] = (rowok && ok) ? (double)ar[u] : 0.0;
      x0[u] = (c0ok && ok) ? (double)b0[u] : 0.0;
      x1[u] = (c1ok && ok) ? (double)b1[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; u += 2) {
      a00 = mfma_f64_16x16x4(a[u], x0[u], a00);
      a01 = mfma_f64_16x16x4(a[u + 1], x0[u + 1], a01);
      a10 = mfma_f64_16x16x4(a[u], x1[u], a10);
      a11 = mfma_f64_16x16x4(a[u + 1], x1[u + 1], a11);
    }
  }
  const dbl4 acc0 = a00 + a01, acc1 = a10 + a11;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = i0 + (lane >> 4) + 4 * v;
    if (row >= rows) continue;
    TO* o = out + (int64_t)row * ldo;
    if (c0ok) o[jb0] = (TO)((beta == 0.0 ? 0.0 : beta * (double)o[jb0]) + alpha * acc0[v]);
    if (c1ok) o[jb1] = (TO)((beta == 0.0 ? 0.0 : beta * (double)o[jb1]) + alpha * acc1[v]);
  }
}

// ------------------------------------------------------------------------------------------
// Row-times-matrix product out[i, :] = beta out[i, :] + alpha A[i, 0:K] M[0:K, :] on the FP64
// matrix cores: one 16 x 16 output tile per workgroup, the NW waves take contiguous slices of the
// K steps and their accumulators are added in LDS in wave order.  NW = 16 when there are fewer
// tiles than compute units (tall-skinny products with a few hundred K steps: more loads in
// flight per tile), else 4.  Used for Q C, W D, G V, V S and the projections X - Q (Q^T X).
// ------------------------------------------------------------------------------------------
template <class TA, class TM, class TO, int NW>
__global__ __launch_bounds__(NW * kWave) void k_rowmul(RowmulProblem<TA, TM, TO> pr0, RowmulProblem<TA, TM, TO> pr1) {
  // two independent products in one launch: blockIdx.z picks one (tiles past its grid exit)
  const RowmulProblem<TA, TM, TO>& pr = blockIdx.z == 0 ? pr0 : pr1;
  const int rows = pr.rows, K = pr.K, lda = pr.lda, ldm = pr.ldm, ldo = pr.ldo, w = pr.w;
  const TA* __restrict__ A = pr.A;
  const TM* __restrict__ M = pr.M;
  TO* __restrict__ out = pr.out;
  const double alpha = pr.alpha, beta = pr.beta;
  double* __restrict__ gpart = pr.gpart;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  if (i0 >= rows || j0 >= w) return;  // uniform over the workgroup
  __shared__ double red[NW - 1][kWave][4];
  __shared__ double tile[16][17];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int ia = i0 + (lane & 15), jb = j0 + (lane & 15), kl = lane >> 4;
  const bool rowok = ia < rows, colok = jb < w;
  // out-of-range operands are loaded from a clamped, valid address and replaced by zero
  const TA* arow = A + (int64_t)min(ia, rows - 1) * lda;
  const TM* mcol = M + min(jb, w - 1);
  const int steps = (K + 3) / 4;
  const int per = (steps + NW - 1) / NW;
  const int s0 = wv * per, s1 = min(steps, s0 + per);
  dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  // full batches of kUnroll k-steps (the last one predicated), so a slice's loads all issue together
  for (int st = s0; st < s1; st += kUnroll) {
    // the loads of the batch first, in the operands' own types, then conversion and masking (with
    // a conversion between them the compiler issued each load only after the previous one returned)
    TA ar[kUnroll];
    TM br[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int kc = min((st + u) * 4 + kl, K - 1);
      ar[u] = arow[kc];
      br[u] = mcol[(int64_t)kc * ldm];
    }
    double a[kUnroll], b[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const bool ok = (st + u < s1) && ((st + u) * 4 + kl < K);
      a[u] = (rowok && ok) ? (double)ar[u] : 0.0;
      b[u] = (colok && ok) ? (double)br[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; u += 2) {
      acc0 = mfma_f64_16x16x4(a[u], b[u], acc0);
      acc1 = mfma_f64_16x16x4(a[u + 1], b[u + 1], acc1);
    }
  }
  dbl4 acc = acc0 + acc1;
  acc = reduce_waves<NW>(acc, red);
  if (wv == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = i0 + (lane >> 4) + 4 * v, col = j0 + (lane & 15);
      double val = 0.0;
      if (row < rows && col < w) {
        TO* o = out + (int64_t)row * ldo + col;
        const TO stored = (TO)((beta == 0.0 ? 0.0 : beta * (double)*o) + alpha * acc[v]);
        *o = stored;
        val = (double)stored;
      }
      tile[(lane >> 4) + 4 * v][lane & 15] = val;
    }
  }
  // Optional epilogue (w <= 16, one column tile): the Gram of this tile's 16 output rows,
  // gpart[blockIdx.x][a][b] = sum_i out[i][a] out[i][b], for the CholeskyQR of the product
  if (gpart == nullptr) return;  // uniform
  __syncthreads();
  const int a = threadIdx.x >> 4, b = threadIdx.x & 15;
  if (a < w && b < w) {
    double sacc = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) sacc = fma(tile[i][a], tile[i][b], sacc);
    gpart[(int64_t)blockIdx.x * w * w + a * w + b] = sacc;
  }
}

// ------------------------------------------------------------------------------------------
// Tall-skinny A^T B on the FP64 matrix cores, split over rows: workgroup (x, y, s) computes the
// 16 x 16 tile (a0, b0) of partial[s] = sum_{i in split s} A[i, :]^T B[i, :] (row stride ldp,
// sstride apart); the NW waves take contiguous slices of the split's rows and are added in wave
// order.  With several splits k_tn_finish (or the consumer) adds them; up to a few thousand rows
// one split of sixteen waves per tile writes the result directly.
// ------------------------------------------------------------------------------------------
template <class TA, class TB, int NW>
__global__ __launch_bounds__(NW * kWave) void k_tn_narrow(int rows, const TA* __restrict__ A, int lda, int na,
                                                          const TB* __restrict__ B, int ldb, int nb,
                                                          double* __restrict__ partial, int64_t sstride, int ldp,
                                                          int rows_per_split) {
  __shared__ double red[NW - 1][kWave][4];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16, s = blockIdx.z;
  const int i0 = s * rows_per_split, i1 = min(rows, i0 + rows_per_split);
  const int aa = a0 + (lane & 15), bb = b0 + (lane & 15), kl = lane >> 4;
  const bool aok = aa < na, bok = bb < nb;
  const TA* acol = A + min(aa, na - 1);
  const TB* bcol = B + min(bb, nb - 1);
  const int steps = (max(i1 - i0, 0) + 3) / 4;
  const int per = (steps + NW - 1) / NW;
  const int s0 = wv * per, s1 = min(steps, s0 + per);
  dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int st = s0; st < s1; st += kUnroll) {  // full batches, the last one predicated
    double a[kUnroll], b[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int row = i0 + (st + u) * 4 + kl;
      const bool ok = (st + u < s1) && (row < i1);
      const int rc = min(row, i1 - 1);
      const double av = (double)acol[(int64_t)rc * lda], bv = (double)bcol[(int64_t)rc * ldb];
      a[u] = (ok && aok) ? av : 0.0;
      b[u] = (ok && bok) ? bv : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; u += 2) {
      acc0 = mfma_f64_16x16x4(a[u], b[u], acc0);
      acc1 = mfma_f64_16x16x4(a[u + 1], b[u + 1], acc1);
    }
  }
  dbl4 acc = acc0 + acc1;
  acc = reduce_waves<NW>(acc, red);
  if (wv == 0) {
    double* P = partial + (int64_t)s * sstride;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ra = a0 + (lane >> 4) + 4 * v, cb = b0 + (lane & 15);
      if (ra < na && cb < nb) P[(int64_t)ra * ldp + cb] = acc[v];
    }
  }
}

__global__ void k_tn_finish(const double* __restrict__ partial, int splits, int na, int nb, double* __restrict__ out,
                            int ldo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)na * nb) return;
  const int a = (int)(t / nb), b = (int)(t % nb);
  double v = 0.0;
  v = split_sum(partial + (int64_t)a * nb + b, splits, (int64_t)na * nb);
  out[(int64_t)a * ldo + b] = v;
}

// ------------------------------------------------------------------------------------------
// Gram G = A^T A (na x na, double) for a tall A on the FP64 matrix cores: one 16 x 16 tile of the
// upper triangle per workgroup, written to both triangles; no partial sums.  The workgroup's 16
// waves take contiguous sixteenths of the rows, and their accumulators are added in wave order
// in LDS (deterministic).  With a few hundred columns there are a few hundred tiles: small tiles
// spread them over every CU, and the row split keeps sixteen streams of loads in flight per tile.
// ------------------------------------------------------------------------------------------
constexpr int kGT = 16;
constexpr int kGramWaves = 16;

template <class T>
__global__ __launch_bounds__(kGramWaves * kWave) void k_gram_tiles(int rows, const T* __restrict__ A, int lda, int na,
                                                                   double* __restrict__ G, int ldg, int ntile) {
  __shared__ double red[kGramWaves - 1][4][kWave];
  // map blockIdx.x to an upper-triangular tile pair (ti <= tj)
  int t = blockIdx.x, ti = 0;
  while (t >= ntile - ti) {
    t -= ntile - ti;
    ++ti;
  }
  const int tj = ti + t;
  const int lane = threadIdx.x & (kWave - 1), grp = threadIdx.x / kWave;
  const int a0 = ti * kGT, b0 = tj * kGT;
  const int aa = a0 + (lane & 15), bb = b0 + (lane & 15), kl = lane >> 4;
  const bool aok = aa < na, bok = bb < na;
  const T* acol = A + min(aa, na - 1);
  const T* bcol = A + min(bb, na - 1);
  const int steps = (rows + 3) / 4;
  const int per = (steps + kGramWaves - 1) / kGramWaves;
  const int s0 = grp * per, s1 = min(steps, s0 + per);
  dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int st = s0; st < s1; st += kUnroll) {
    double a[kUnroll], b[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int row = (st + u) * 4 + kl;
      const bool ok = (st + u < s1) && (row < rows);
      const int rc = min(row, rows - 1);
      const double av = (double)acol[(int64_t)rc * lda], bv = (double)bcol[(int64_t)rc * lda];
      a[u] = (ok && aok) ? av : 0.0;
      b[u] = (ok && bok) ? bv : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; u += 2) {
      acc0 = mfma_f64_16x16x4(a[u], b[u], acc0);
      acc1 = mfma_f64_16x16x4(a[u + 1], b[u + 1], acc1);
    }
  }
  dbl4 acc = acc0 + acc1;
  if (grp > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) red[grp - 1][v][lane] = acc[v];
  }
  __syncthreads();
  if (grp > 0) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double sum = acc[v];
    for (int g = 0; g < kGramWaves - 1; ++g) sum += red[g][v][lane];
    const int ra = a0 + (lane >> 4) + 4 * v, cb = b0 + (lane & 15);
    if (ra < na && cb < na) {
      G[(int64_t)ra * ldg + cb] = sum;
      if (ti != tj) G[(int64_t)cb * ldg + ra] = sum;
    }
  }
}

// The same Gram with 32 x 32 tiles, for blocks of several hundred columns: each wave holds the
// tile as 2 x 2 matrix-instruction blocks, so a k-step loads two 64-byte segments per side and
// issues four independent products (twice the products per load of the 16 x 16 tiles, and a
// quarter of the workgroups re-reading A).  Eight waves split the rows.
constexpr int kGT2 = 32;
constexpr int kGram2Waves = 8;
constexpr int kGram32MinCols = 416;  // measured crossover with the 16 x 16 tiles (1024 and 3706 rows)

template <class T>
__global__ __launch_bounds__(kGram2Waves * kWave) void k_gram_tiles32(int rows, const T* __restrict__ A, int lda,
                                                                      int na, double* __restrict__ G, int ldg,
                                                                      int ntile) {
  __shared__ double red[kGram2Waves - 1][16][kWave];
  int t = blockIdx.x, ti = 0;
  while (t >= ntile - ti) {
    t -= ntile - ti;
    ++ti;
  }
  const int tj = ti + t;
  const bool diag = ti == tj;
  const int lane = threadIdx.x & (kWave - 1), grp = threadIdx.x / kWave;
  const int a0 = ti * kGT2, b0 = tj * kGT2;
  const int c = lane & 15, kl = lane >> 4;
  // Columns past na are read at column na - 1: a lane's A operand only reaches output row
  // a0 + 16 i + c and its B operand only output column b0 + 16 j + c, which are not stored.
  const T* acol[2];
  const T* bcol[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    acol[h] = A + min(a0 + 16 * h + c, na - 1);
    bcol[h] = A + min(b0 + 16 * h + c, na - 1);
  }
  const int steps = (rows + 3) / 4;
  const int per = (steps + kGram2Waves - 1) / kGram2Waves;
  const int s0 = grp * per, s1 = min(steps, s0 + per);
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  auto batch = [&](int st, bool tail) {
    double a[kUnroll][2], b[kUnroll][2];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int row = (st + u) * 4 + kl;
      const int64_t off = (int64_t)(tail ? min(row, rows - 1) : row) * lda;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        a[u][h] = (double)acol[h][off];
        b[u][h] = (double)bcol[h][off];
      }
      // rows past this wave's range or past the end add nothing (a zero A operand)
      if (tail && !((st + u < s1) && (row < rows))) a[u][0] = a[u][1] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f64_16x16x4(a[u][i], b[u][j], acc[i][j]);
  };
  int st = s0;
  // full batches: every row of the batch lies in this wave's range and in A
  for (; st + kUnroll <= s1 && (st + kUnroll) * 4 <= rows; st += kUnroll) batch(st, false);
  for (; st < s1; st += kUnroll) batch(st, true);
  if (grp > 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[grp - 1][(i * 2 + j) * 4 + v][lane] = acc[i][j][v];
  }
  __syncthreads();
  if (grp > 0) return;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double sum = acc[i][j][v];
        for (int g = 0; g < kGram2Waves - 1; ++g) sum += red[g][(i * 2 + j) * 4 + v][lane];
        const int ra = a0 + 16 * i + kl + 4 * v, cb = b0 + 16 * j + c;
        if (ra < na && cb < na) {
          G[(int64_t)ra * ldg + cb] = sum;
          if (!diag) G[(int64_t)cb * ldg + ra] = sum;
        }
      }
}

// ------------------------------------------------------------------------------------------
// Reductions (double accumulation)
// ------------------------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_sumsq_cols(int rows, const T* __restrict__ A, int lda, int c0, int w,
                                                    double* __restrict__ partial) {
  __shared__ double lds[4];
  double v = 0.0;
  const int64_t total = (int64_t)rows * w;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / w), c = (int)(e % w);
    const double x = (double)A[(int64_t)i * lda + c0 + c];
    v = fma(x, x, v);
  }
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <class T>
__global__ __launch_bounds__(256) void k_sumsq(int64_t len, const T* __restrict__ x, double* __restrict__ partial) {
  __shared__ double lds[4];
  double v = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
    const double xe = (double)x[e];
    v = fma(xe, xe, v);
  }
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// scal[slot + q] = sum_b partial[b * stride + q] for q < nq: one workgroup, each thread sums a
// fixed strided subset, then a fixed butterfly and wave order (deterministic).
__global__ __launch_bounds__(256) void k_finish(const double* __restrict__ partial, int nblocks, int stride, int nq,
                                                double* scal, int slot, const double* post_src, int post_count,
                                                double* post_dst, unsigned* post_flag, unsigned post_seq) {
  __shared__ double lds[4];
  for (int q = 0; q < nq; ++q) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += partial[(int64_t)b * stride + q];
    const double t = block_sum(v, lds);
    if (threadIdx.x == 0) scal[slot + q] = t;
  }
  if (post_dst != nullptr) post_to_host(post_src, post_count, post_dst, post_flag, post_seq);  // uniform
}

__global__ void k_diag_sqrt(const double* __restrict__ G, int ldg, int w, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < w) out[c] = sqrt(fmax(G[(int64_t)c * ldg + c], 0.0));
}

constexpr int kBlockCholThreads = 1024;

// ------------------------------------------------------------------------------------------
// Cholesky factor of a block's Gram (CholeskyQR with column dropping), one workgroup, double.
// Input: the w x w Gram of the projected block and the column norms before projection.
// A column c is dropped when its projected norm is at most drop_tol * prenorm[c] (it lies in
// the span of the basis it was projected against; skipped when prenorm == nullptr), or when
// its Cholesky pivot is at most dep_tol times its projected norm (it depends on the kept
// columns before it; a Gram-based pivot cannot resolve dependence much below 1e-8).  The
// factor R (upper, R^T R = Gram of the kept columns) goes to Rout for k_trsm_rows, which writes
// X_new = X[:, kept] R^{-1}: wk orthonormal columns followed by zero columns.  If wk_in >= 0
// only the first wk_in columns take part (second pass of CholeskyQR2 reads the count of the
// first pass from scal[wk_slot_in]).  scal[slot] = wk.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlockCholThreads) void k_block_chol(const double* __restrict__ gram, int ldg,
                                                                  int splits, int64_t sstride, int w,
                                                                  const double* __restrict__ prenorm, double drop_tol,
                                                                  double dep_tol, double* __restrict__ Rout, int ldm,
                                                                  double* scal, int slot, int wk_slot_in) {
  extern __shared__ double sm[];
  const int ld = w + 1;
  double* A = sm;  // w x (w + 1): Gram, overwritten by the Schur complements / rows of R
  __shared__ int keep[kEigMax];
  __shared__ double gdiag[kEigMax];
  // a 32 x 32 grid of threads: row ty, column tx
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  int wa = w;
  if (wk_slot_in >= 0) wa = min(w, (int)scal[wk_slot_in]);
  // the Gram is the sum of `splits` partial Grams (sstride apart), added in a fixed order
  for (int i = ty; i < w; i += 32)
    for (int j = tx; j < w; j += 32) {
      double v = 0.0;
      if (i < wa && j < wa) v = split_sum(gram + (int64_t)i * ldg + j, splits, sstride);
      A[i * ld + j] = v;
    }
  __syncthreads();
  for (int c = tid; c < w; c += blockDim.x) {
    const double g = (c < wa) ? fmax(A[c * ld + c], 0.0) : 0.0;
    gdiag[c] = g;
    const double lim = prenorm ? drop_tol * prenorm[c] : 0.0;
    keep[c] = (c < wa) && (sqrt(g) > lim) ? 1 : 0;
  }
  __syncthreads();
  // Right-looking Cholesky on the upper triangle.  At step c every thread reads the pivot
  // d = A[c][c] (the Schur complement) and takes the same keep decision; a kept column then
  // updates the trailing upper triangle A[i][j] -= A[c][i] A[c][j] / d, i, j > c.  The decision
  // is uniform, so a step without an update needs no barrier, and keep[c] (read only after the
  // loop) is cleared without one.
  for (int c = 0; c < wa; ++c) {
    if (!keep[c]) continue;  // uniform: keep[c] is only written at step c itself
    const double d = A[c * ld + c];
    const bool ok = (d > dep_tol * dep_tol * gdiag[c]) && (d > 0.0);
    if (!ok) {
      if (tid == 0) keep[c] = 0;
      continue;
    }
    const double inv = 1.0 / d;
    for (int i = c + 1 + ty; i < wa; i += 32) {
      const double aci = A[c * ld + i];
      for (int j = c + 1 + tx; j < wa; j += 32)
        if (i <= j) A[i * ld + j] -= aci * A[c * ld + j] * inv;
    }
    __syncthreads();
  }
  __syncthreads();
  // Rout: row c of the factor for kept c (R[c][c] = sqrt(pivot), R[c][j] = A[c][j] / R[c][c]);
  // a dropped column keeps an all-zero row and column, R[c][c] = 0 marking it for the row solve.
  for (int c = ty; c < w; c += 32)
    for (int j = tx; j < w; j += 32) {
      double v = 0.0;
      if (c < wa && j < wa && j >= c && keep[c] && keep[j]) {
        const double rc = sqrt(A[c * ld + c]);
        v = (j == c) ? rc : A[c * ld + j] / rc;
      }
      Rout[(int64_t)c * ldm + j] = v;
    }
  if (tid == 0) {
    int q = 0;
    for (int c = 0; c < wa; ++c) q += keep[c];
    scal[slot] = (double)q;
  }
}

// ------------------------------------------------------------------------------------------
// Row-wise solve Z R = X for the factor of k_block_chol: one thread per row, forward
// substitution in double over the columns with R broadcast from LDS; the kept columns are
// written packed to the left of out and the remaining columns are zero.
// ------------------------------------------------------------------------------------------
template <int WM, class T>
__global__ __launch_bounds__(256) void k_trsm_rows(int rows, const T* __restrict__ X, int ldx, int w,
                                                   const double* __restrict__ R, int ldr, T* __restrict__ out,
                                                   int ldo) {
  extern __shared__ double Rs[];  // w x (w + 1)
  const int ld = w + 1;
  for (int e = threadIdx.x; e < w * w; e += blockDim.x) Rs[(e / w) * ld + e % w] = R[(int64_t)(e / w) * ldr + e % w];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  // loads first (columns clamped to w - 1, w >= 1), then conversion and masking, so they issue together
  T xr[WM];
#pragma unroll
  for (int c = 0; c < WM; ++c) xr[c] = X[(int64_t)i * ldx + min(c, w - 1)];
  double z[WM];
#pragma unroll
  for (int c = 0; c < WM; ++c) z[c] = (c < w) ? (double)xr[c] : 0.0;
#pragma unroll
  for (int c = 0; c < WM; ++c) {
    if (c < w) {
      double v = z[c];
#pragma unroll
      for (int l = 0; l < c; ++l) v = fma(-z[l], Rs[l * ld + c], v);
      const double rcc = Rs[c * ld + c];
      z[c] = (rcc != 0.0) ? v / rcc : 0.0;
    }
  }
  T* o = out + (int64_t)i * ldo;
  int q = 0;
#pragma unroll
  for (int c = 0; c < WM; ++c) {
    if (c < w && Rs[c * ld + c] != 0.0) o[q++] = (T)z[c];
  }
  for (; q < w; ++q) o[q] = (T)0;
}

// ------------------------------------------------------------------------------------------
// One CholeskyQR pass in one launch: every one-wave workgroup adds the Gram partials (in a fixed
// order), factors the Gram with the column-drop rules of k_block_chol in LDS (the same pivots,
// decisions and factor in every workgroup), and solves its 64 rows as k_trsm_rows does:
// out = X[:, kept] R^{-1}, kept columns packed left, zeros after them.  The factorisation is
// repeated per workgroup (w^3 / 6 flops) instead of being a launch of its own.  With gout, each
// workgroup also writes the Gram of its 64 stored output rows (gout[blockIdx.x], w x w), so a
// second pass needs no separate Gram launch.  Workgroup 0 writes the kept count to scal[slot];
// with wk_slot_in >= 0 only the first scal[wk_slot_in] columns take part (second pass).
// ------------------------------------------------------------------------------------------
constexpr int kCholTrsmRows = 64;      // rows solved per workgroup
constexpr int kCholTrsmThreads = 256;  // threads that load and factor the Gram (a 16 x 16 grid)

template <int WM, class T>
__global__ __launch_bounds__(kCholTrsmThreads) void k_chol_trsm(int rows, const T* __restrict__ X, int ldx, int w,
                                                             const double* __restrict__ gram, int splits,
                                                             int64_t sstride, const double* __restrict__ prenorm,
                                                             double drop_tol, double dep_tol, int wk_slot_in,
                                                             T* __restrict__ out, int ldo, double* __restrict__ gout,
                                                             double* scal, int slot) {
  constexpr int ld = WM + 1;
  constexpr int kPer = WM * WM / kCholTrsmThreads;  // entries of the WM x WM square per thread
  __shared__ double A[WM * ld];             // Gram, Schur complements, then the rows of R
  __shared__ double O[kCholTrsmRows][ld];   // stored output rows (for gout)
  __shared__ int keep[WM];
  __shared__ double gdiag[WM], rdiag[WM], rinv[WM];
  const int tid = threadIdx.x;
  int wa = w;
  if (wk_slot_in >= 0) wa = min(w, (int)scal[wk_slot_in]);
  // the Gram is the sum of `splits` partial Grams (w x w, sstride apart), added in a fixed order;
  // entry (i, j) of the WM x WM square is e = i WM + j (compile-time shifts, no division)
  if (splits == 1) {  // uniform: one Gram, every entry's load in flight at once
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * kCholTrsmThreads, i = e / WM, j = e % WM;
      A[i * ld + j] = (i < wa && j < wa) ? gram[i * w + j] : 0.0;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * kCholTrsmThreads, i = e / WM, j = e % WM;
      A[i * ld + j] = (i < wa && j < wa) ? split_sum(gram + i * w + j, splits, sstride) : 0.0;
    }
  }
  __syncthreads();
  for (int c = tid; c < w; c += kCholTrsmThreads) {
    const double g = (c < wa) ? fmax(A[c * ld + c], 0.0) : 0.0;
    gdiag[c] = g;
    const double lim = prenorm ? drop_tol * prenorm[c] : 0.0;
    keep[c] = (c < wa) && (sqrt(g) > lim) ? 1 : 0;
  }
  __syncthreads();
  // right-looking Cholesky on the upper triangle (k_block_chol's order and decisions).  Up to 32
  // columns each thread owns fixed entries of the square (unrolled); wider blocks spread the
  // trailing triangle over a 16 x 16 grid of threads.  The keep decision is uniform: a step without
  // an update needs no barrier, and keep[c] (read only after the loop) is cleared without one.
  if constexpr (WM <= 32) {
    for (int c = 0; c < wa; ++c) {
      if (!keep[c]) continue;  // uniform
      const double d = A[c * ld + c];
      const bool ok = (d > dep_tol * dep_tol * gdiag[c]) && (d > 0.0);
      if (ok) {
        const double inv = rcp_nr(d);
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
          const int e = tid + k * kCholTrsmThreads, i = e / WM, j = e % WM;
          if (i > c && i <= j && j < wa) A[i * ld + j] -= A[c * ld + i] * A[c * ld + j] * inv;
        }
      }
      __syncthreads();
      if (!ok && tid == 0) keep[c] = 0;
      __syncthreads();
    }
  } else {
    const int tx = tid & 15, ty = tid >> 4;
    for (int c = 0; c < wa; ++c) {
      if (!keep[c]) continue;  // uniform: keep[c] is only written at step c itself
      const double d = A[c * ld + c];
      const bool ok = (d > dep_tol * dep_tol * gdiag[c]) && (d > 0.0);
      if (!ok) {
        if (tid == 0) keep[c] = 0;
        continue;
      }
      const double inv = rcp_nr(d);
      for (int i = c + 1 + ty; i < wa; i += 16) {
        const double aci = A[c * ld + i];
        for (int j = c + 1 + tx; j < wa; j += 16)
          if (i <= j) A[i * ld + j] -= aci * A[c * ld + j] * inv;
      }
      __syncthreads();
    }
    __syncthreads();
  }
  // rows of R in place: R[c][c] = sqrt(pivot), R[c][j] = A[c][j] / R[c][c] (j > c); zero rows and
  // columns for the dropped and inactive indices
  for (int c = tid; c < WM; c += kCholTrsmThreads) {
    const bool kc = c < wa && keep[c];
    const double ri = kc ? rsq_nr(A[c * ld + c]) : 0.0;  // 1 / R[c][c]
    rinv[c] = ri;
    rdiag[c] = kc ? A[c * ld + c] * ri : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int e = tid + k * kCholTrsmThreads, c = e / WM, j = e % WM;
    double v = 0.0;
    if (j >= c && rdiag[c] != 0.0 && rdiag[j] != 0.0) v = (j == c) ? rdiag[c] : A[c * ld + j] * rinv[c];
    A[c * ld + j] = v;
  }
  __syncthreads();
  // forward substitution of this thread's row
  if constexpr (WM > 32) {
    // Wide blocks: the workgroup's 64 rows are solved in 16-column panels.  The rows sit in O as
    // double; for panel J the update from the solved panels, O[:, J] -= O[:, <J] R[<J, J], runs on
    // the matrix cores (wave v: rows 16 v .. 16 v + 15), and only the panel's own 16 x 16 triangle
    // is solved row by row.  Kept columns are then written packed to the left of out.
    static_assert(WM % 16 == 0 && kCholTrsmRows == 64 && kCholTrsmThreads == 256, "four waves of 16 rows");
    const int row0 = blockIdx.x * kCholTrsmRows;
    for (int e = tid; e < kCholTrsmRows * WM; e += kCholTrsmThreads) {
      const int r = e / WM, c = e % WM, gi = row0 + r;
      O[r][c] = (gi < rows && c < w) ? (double)X[(int64_t)gi * ldx + c] : 0.0;
    }
    __syncthreads();
    const int lane = tid & (kWave - 1), wv = tid / kWave;
    for (int c0 = 0; c0 < w; c0 += 16) {
      if (c0 > 0) {
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < c0; k0 += 4) {
          const double a = O[16 * wv + (lane & 15)][k0 + (lane >> 4)];
          const double b = A[(k0 + (lane >> 4)) * ld + c0 + (lane & 15)];
          acc = mfma_f64_16x16x4(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) O[16 * wv + (lane >> 4) + 4 * v][c0 + (lane & 15)] -= acc[v];
        __syncthreads();
      }
      if (tid < kCholTrsmRows) {
        // the panel's 16 values of this row in registers (columns past w are zero and stay zero)
        double z[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) z[c] = O[tid][c0 + c];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          double v = z[c];
#pragma unroll
          for (int l = 0; l < c; ++l) v = fma(-z[l], A[(c0 + l) * ld + c0 + c], v);
          z[c] = v * rinv[c0 + c];  // 0 for a dropped column
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) O[tid][c0 + c] = z[c];
      }
      __syncthreads();
    }
    if (tid < kCholTrsmRows) {
      const int i = row0 + tid;
      const bool live = i < rows;
      int q = 0;
      for (int c = 0; c < w; ++c) {
        if (A[c * ld + c] != 0.0) {
          if (live) out[(int64_t)i * ldo + q] = (T)O[tid][c];
          ++q;
        }
      }
      for (int c = q; c < w; ++c)
        if (live) out[(int64_t)i * ldo + c] = (T)0;
      if (blockIdx.x == 0 && tid == 0) scal[slot] = (double)q;
    }
    return;  // no Gram of the output for wide blocks (gout is for at most 32 columns)
  }
  // the first wave solves the workgroup's 64 rows, one per lane
  if (tid >= kCholTrsmRows) return;
  const int i = blockIdx.x * kCholTrsmRows + tid;
  const bool live = i < rows;
  // the row's loads first (clamped, valid addresses: rows, w >= 1), then conversion and masking; with
  // a masked conversion per load the compiler issued each load only after the previous one returned
  T xr[WM];
  const T* xrow = X + (int64_t)min(i, rows - 1) * ldx;
#pragma unroll
  for (int c = 0; c < WM; ++c) xr[c] = xrow[min(c, w - 1)];
  double z[WM];
#pragma unroll
  for (int c = 0; c < WM; ++c) z[c] = (live && c < w) ? (double)xr[c] : 0.0;
#pragma unroll
  for (int c = 0; c < WM; ++c) {
    if (c < w) {
      double v = z[c];
#pragma unroll
      for (int l = 0; l < c; ++l) v = fma(-z[l], A[l * ld + c], v);
      z[c] = v * rinv[c];  // 0 for a dropped column
    }
  }
  int q = 0;
#pragma unroll
  for (int c = 0; c < WM; ++c) {
    if (c < w && A[c * ld + c] != 0.0) {
      const T t = (T)z[c];
      if (live) out[(int64_t)i * ldo + q] = t;
      O[tid][q] = live ? (double)t : 0.0;
      ++q;
    }
  }
  for (int c = q; c < w; ++c) {
    if (live) out[(int64_t)i * ldo + c] = (T)0;
    O[tid][c] = 0.0;
  }
  if (blockIdx.x == 0 && tid == 0) scal[slot] = (double)q;
  if (gout == nullptr) return;  // uniform
  __builtin_amdgcn_wave_barrier();  // one wave from here: its LDS writes are visible to its reads
  // Gram of the 64 stored rows on the FP64 matrix cores: 16 x 16 tiles (ta, tb), lane l takes
  // rows 4 s + l / 16 of columns l % 16; the result holds rows (l / 16) + 4 v of column l % 16
  const int nt = (w + 15) / 16, lane = tid, kl = lane >> 4, cl = lane & 15;
  double* go = gout + (int64_t)blockIdx.x * w * w;
  for (int t = 0; t < nt * nt; ++t) {
    const int ta = t / nt, tb = t % nt;
    const int ca = ta * 16 + cl, cb = tb * 16 + cl;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < kCholTrsmRows / 4; ++st) {
      const int r = st * 4 + kl;
      const double av = (ca < w) ? O[r][ca] : 0.0, bv = (cb < w) ? O[r][cb] : 0.0;
      acc = mfma_f64_16x16x4(av, bv, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ra = ta * 16 + kl + 4 * v, cbo = tb * 16 + cl;
      if (ra < w && cbo < w) go[ra * w + cbo] = acc[v];
    }
  }
}

// 16-byte vectors of the storage type and their dot product, element by element in order
template <class T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};
__device__ inline float dot16(Vec16<float>::type a, Vec16<float>::type b, float x) {
  x = fmaf(a.x, b.x, x);
  x = fmaf(a.y, b.y, x);
  x = fmaf(a.z, b.z, x);
  return fmaf(a.w, b.w, x);
}
__device__ inline double dot16(Vec16<double>::type a, Vec16<double>::type b, double x) {
  x = fma(a.x, b.x, x);
  return fma(a.y, b.y, x);
}

// ------------------------------------------------------------------------------------------
// Fused sampled product and dual update on Lambda (CSC order), Eq. 4 with X = Ut Vt^T:
//   x = <Ut[i,:], Vt[j,:]>, res = a - x, y_next = y + delta res, sums of res^2, y_next^2, |res|.
// Work comes in chunks of at most kSddmmChunk consecutive CSC positions of one column (the chunk
// table is built once at set-up), one wave per chunk, so power-law columns do not serialise on
// one wave.  Vt[j, :] is staged in LDS.  The dot product and the update run in T; the sums
// accumulate in double.  With yT set, y_next also goes to the dense transposed copy of the
// iterate (yT[j * ldy + i]), which the next R4SVD call's products then read as they are.
// KB (1, 2, 4 or 8) is the batch of factor vectors per row whose loads are in flight together.
// ------------------------------------------------------------------------------------------
template <class T, int KB>
__global__ __launch_bounds__(256) void k_sddmm_update(int nchunks, const int32_t* __restrict__ cstart,
                                                      const int32_t* __restrict__ ccol,
                                                      const int32_t* __restrict__ rowidx, const T* __restrict__ a,
                                                      const T* __restrict__ y, T* __restrict__ y_next,
                                                      const T* __restrict__ Ut, const T* __restrict__ Vt, int ld,
                                                      int k, T delta, double* __restrict__ partial,
                                                      T* __restrict__ yT, int64_t ldy) {
  using V = typename Vec16<T>::type;  // 16-byte vector of T
  constexpr int E = Vec16<T>::n;
  extern __shared__ __align__(16) unsigned char sdd_lds[];
  __shared__ double lds[4];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int c = blockIdx.x * 4 + wid;
  const int kv = (k + E - 1) / E;  // 16-byte vectors per factor row (ld is a multiple of E)
  T* vsw = reinterpret_cast<T*>(sdd_lds) + (size_t)wid * kv * E;  // this wave's row of Vt
  double s_res = 0.0, s_y = 0.0, s_abs = 0.0;
  int p0 = 0, p1 = 0, j = 0;
  if (c < nchunks) {
    p0 = cstart[c];
    p1 = cstart[c + 1];
    j = ccol[c];
    // Vt[j, :k] and zeros up to the vector boundary (the factor buffers are zero-initialised, so
    // the padded products are exact zeros)
    for (int l = lane; l < kv * E; l += kWave) vsw[l] = (l < k) ? Vt[(int64_t)j * ld + l] : (T)0;
  }
  __syncthreads();
  const V* vv = reinterpret_cast<const V*>(vsw);
  T* ycol = yT ? yT + (int64_t)j * ldy : nullptr;
  auto update = [&](int p, int i, T x) {
    const T res = a[p] - x;
    const T yn = fma(delta, res, y[p]);
    y_next[p] = yn;
    if (ycol) ycol[i] = yn;
    s_res = fma((double)res, (double)res, s_res);
    s_y = fma((double)yn, (double)yn, s_y);
    s_abs += fabs((double)res);
  };
  // The factor rows go in batches of kB vectors with every load of a batch in flight before its
  // products: indices past kv are clamped to the row's last vector (a valid address) and meet a zero
  // vector of Vt, so the products and their order are those of the plain loop over kv.  (A loop over
  // kv unrolled by the compiler took one memory round trip per vector below its unroll width.)
  constexpr int kB = KB;
  const V vzero = {};
  auto dots = [&](const V* u0, const V* u1, T& x0, T& x1, bool two) {
    for (int l0 = 0; l0 < kv; l0 += kB) {
      V a0[kB], a1[kB], bv[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int l = min(l0 + u, kv - 1);
        a0[u] = u0[l];
        if (two) a1[u] = u1[l];  // uniform
        bv[u] = (l0 + u < kv) ? vv[l] : vzero;
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        x0 = dot16(a0[u], bv[u], x0);
        if (two) x1 = dot16(a1[u], bv[u], x1);
      }
    }
  };
  // two entries per lane and step: both factor rows are in flight before the products
  int p = p0 + lane;
  for (; p + kWave < p1; p += 2 * kWave) {
    const int i0 = rowidx[p], i1 = rowidx[p + kWave];
    const V* u0 = reinterpret_cast<const V*>(Ut + (int64_t)i0 * ld);
    const V* u1 = reinterpret_cast<const V*>(Ut + (int64_t)i1 * ld);
    T x0 = (T)0, x1 = (T)0;
    dots(u0, u1, x0, x1, true);
    update(p, i0, x0);
    update(p + kWave, i1, x1);
  }
  if (p < p1) {
    const int i0 = rowidx[p];
    const V* u0 = reinterpret_cast<const V*>(Ut + (int64_t)i0 * ld);
    T x0 = (T)0, x1 = (T)0;
    dots(u0, u0, x0, x1, false);
    update(p, i0, x0);
  }
  const double t0 = block_sum(s_res, lds);
  const double t1 = block_sum(s_y, lds);
  const double t2 = block_sum(s_abs, lds);
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x] = t0;
    partial[3 * blockIdx.x + 1] = t1;
    partial[3 * blockIdx.x + 2] = t2;
  }
}

// partial[b] = sum over this block's entries of |ref - x| (double), grid-stride
__global__ __launch_bounds__(256) void k_absdiff(int64_t len, const double* __restrict__ x,
                                                 const double* __restrict__ ref, double* __restrict__ partial) {
  __shared__ double lds[4];
  double v = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x)
    v += fabs(ref[e] - x[e]);
  const double t = block_sum(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

template <class T>
__global__ void k_sample(int64_t nq, const int32_t* __restrict__ qi, const int32_t* __restrict__ qj,
                         const T* __restrict__ Ut, const T* __restrict__ Vt, int ld, int k, int64_t m, int64_t n,
                         double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nq) return;
  const int32_t i = qi[t], j = qj[t];
  if (i < 0 || i >= m || j < 0 || j >= n) {  // an index outside the matrix reads nothing and yields NaN
    out[t] = __builtin_nan("");
    return;
  }
  const T* u = Ut + (int64_t)i * ld;
  const T* v = Vt + (int64_t)j * ld;
  T x = (T)0;
  for (int l = 0; l < k; ++l) x = fma(u[l], v[l], x);
  out[t] = (double)x;
}

// Per-block sums of |ref - X(qi, qj)| over a grid-stride loop: X as k_sample computes it and the
// sum in the order of k_absdiff, so the total equals sample-then-absdiff bit for bit.  An index out
// of range contributes NaN (no read happens), which makes the result NaN.
template <class T>
__global__ __launch_bounds__(256) void k_sample_absdiff(int64_t nq, const int32_t* __restrict__ qi,
                                                        const int32_t* __restrict__ qj, const T* __restrict__ Ut,
                                                        const T* __restrict__ Vt, int ld, int k, int64_t m,
                                                        int64_t n, const double* __restrict__ ref,
                                                        double* __restrict__ partial) {
  __shared__ double lds[4];
  double v = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nq; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = qi[e], j = qj[e];
    if (i < 0 || i >= m || j < 0 || j >= n) {
      v += __builtin_nan("");
      continue;
    }
    const T* u = Ut + (int64_t)i * ld;
    const T* w = Vt + (int64_t)j * ld;
    T x = (T)0;
    for (int l = 0; l < k; ++l) x = fma(u[l], w[l], x);
    v += fabs(ref[e] - (double)x);
  }
  const double t = block_sum(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// dst[0] = src[0] / denom
__global__ void k_div_store(const double* __restrict__ src, double denom, double* __restrict__ dst) {
  if (threadIdx.x == 0) dst[0] = src[0] / denom;
}

template <class TS, class TD>
__global__ void k_scale_copy(int64_t len, const TS* __restrict__ src, double alpha, TD* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < len) dst[t] = (TD)(alpha * (double)src[t]);
}

// dst[t] = src[perm[t]]: a vector on Lambda from the library's CSC order back to the caller's order
__global__ void k_gather_perm(int64_t len, const int32_t* __restrict__ perm, const double* __restrict__ src,
                              double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < len) dst[t] = src[perm[t]];
}

template <class TS, class TD>
__global__ void k_copy_cols(int rows, const TS* __restrict__ src, int lds_, TD* __restrict__ dst, int ldd, int w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * w) return;
  const int i = (int)(t / w), c = (int)(t % w);
  dst[(int64_t)i * ldd + c] = (TD)src[(int64_t)i * lds_ + c];
}

inline unsigned grid1(int64_t work, int per = 256) { return (unsigned)((work + per - 1) / per); }

}  // namespace

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
int tiled_row_tiles(int64_t m) { return (int)((m + kTR - 1) / kTR); }

template <class T>
hipError_t launch_omega(hipStream_t s, T* om, int n, int c0, int w, int ld, uint64_t seed, uint64_t blk,
                        uint64_t it) {
  const int64_t work = (int64_t)n * ((w + 3) / 4);
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL(k_omega<T>, dim3(grid1(work)), dim3(256), 0, s, om, n, c0, w, ld, seed, blk, it);
  return hipGetLastError();
}

hipError_t launch_fill_random(hipStream_t s, double* V, int rows, int ld, int c0, int c1, uint64_t seed,
                              uint64_t tag) {
  const int64_t work = (int64_t)rows * (c1 - c0);
  if (work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_random, dim3(grid1(work)), dim3(256), 0, s, V, rows, ld, c0, c1, seed, tag);
  return hipGetLastError();
}

hipError_t launch_set_unit(hipStream_t s, double* V, int rows, int ld, int c0, int count, int row0) {
  const int64_t work = (int64_t)rows * count;
  if (work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_unit, dim3(grid1(work)), dim3(256), 0, s, V, rows, ld, c0, count, row0);
  return hipGetLastError();
}

template <class T, class TD>
hipError_t launch_seg_spmm(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* vperm,
                           const T* val, const TD* D, int ldd, T* out, int ldo, int w, int64_t total, int max_len,
                           const SegChunks* ch) {
  if (nrows == 0 || w == 0) return hipSuccess;
  constexpr int CPL = 4;
  const unsigned gy = (unsigned)((w + kWave * CPL - 1) / (kWave * CPL));
  const bool vec = rows_vec4(D, ldd);
  // one wave per segment: segments [ptr[q], ptr[q+1]) or, with lo given, [lo[q], hi[q]); narrow
  // blocks give a whole workgroup to each segment when segments average 256 positions or more
  auto segments = [&](int nseg, T* o, int ldo_, const int32_t* lo, const int32_t* hi, const int32_t* skip,
                      bool long_segments) {
    const unsigned gx = (unsigned)((nseg + 3) / 4);
    if (w <= kNarrow && long_segments)
      hipLaunchKernelGGL((k_seg_spmm_narrow<kNarrow, 4, T, TD>), dim3(nseg), dim3(256), 0, s, nseg, ptr, idx, vperm, val,
                         D, ldd, o, ldo_, w, lo, hi, skip);
    else if (w <= kNarrow)
      hipLaunchKernelGGL((k_seg_spmm_narrow<kNarrow, 1, T, TD>), dim3(gx), dim3(256), 0, s, nseg, ptr, idx, vperm, val,
                         D, ldd, o, ldo_, w, lo, hi, skip);
    else if (vec)
      hipLaunchKernelGGL((k_seg_spmm_wide<CPL, true, T, TD>), dim3(gx, gy), dim3(256), 0, s, nseg, ptr, idx, vperm, val,
                         D, ldd, o, ldo_, w, lo, hi, skip);
    else
      hipLaunchKernelGGL((k_seg_spmm_wide<CPL, false, T, TD>), dim3(gx, gy), dim3(256), 0, s, nseg, ptr, idx, vperm, val,
                         D, ldd, o, ldo_, w, lo, hi, skip);
    return hipGetLastError();
  };
  const bool chunked = ch != nullptr && ch->nlong > 0 && w <= ch->ldp;
  hipError_t e = segments(nrows, out, ldo, nullptr, nullptr, chunked ? ch->skip : nullptr,
                          total >= (int64_t)kNarrowSplitLen * nrows ||
                              std::min(max_len, chunked ? kSegLong : max_len) >= kNarrowSplitMax);
  if (e != hipSuccess || !chunked) return e;
  // long segments: one wave per chunk into the partial rows, then the chunks of each segment added in order
  T* P = reinterpret_cast<T*>(ch->P);
  e = segments(ch->nchunk, P, ch->ldp, ch->lo, ch->hi, nullptr, true);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_chunk_sum<T>, dim3((w + 255) / 256, ch->nlong), dim3(256), 0, s, ch->lcol, ch->lfirst, P,
                     ch->ldp, out, ldo, w);
  return hipGetLastError();
}

template <class T, class TQ>
hipError_t launch_spmm_t_tiled(hipStream_t s, int m, int n, const int32_t* rowidx, const int32_t* tstart,
                               const T* val, const TQ* Q, int ldq, int r, T* W, int ldw, double* partial,
                               int64_t partial_cap) {
  if (n == 0 || r == 0) return hipSuccess;
  const int nt = tiled_row_tiles(m);
  const int gx = (n + kTJ - 1) / kTJ, gy = (r + kTC - 1) / kTC;
  int splits = std::max(1, std::min(nt, 512 / std::max(1, gx * gy)));
  while (splits > 1 && (int64_t)splits * n * r > partial_cap) --splits;
  const int tps = (nt + splits - 1) / splits;
  splits = (nt + tps - 1) / tps;
  if (splits == 1) {
    hipLaunchKernelGGL((k_spmm_t_tiled<T, TQ>), dim3(gx, gy, 1), dim3(256), 0, s, m, n, rowidx, tstart, nt, val, Q, ldq, r,
                       W, ldw, tps, (int64_t)0);
    return hipGetLastError();
  }
  T* part = reinterpret_cast<T*>(partial);
  const int64_t stride = (int64_t)n * r;
  hipLaunchKernelGGL((k_spmm_t_tiled<T, TQ>), dim3(gx, gy, splits), dim3(256), 0, s, m, n, rowidx, tstart, nt, val, Q, ldq,
                     r, part, r, tps, stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_split_sum<T>, dim3(grid1((int64_t)n * r)), dim3(256), 0, s, n, r, part, splits, stride, r, W,
                     ldw);
  return hipGetLastError();
}

// 16 x 16 tiles from which a product runs as k_rowmul_tall
constexpr unsigned kTallMinTiles = 2048;

template <class TA, class TM, class TO>
hipError_t launch_rowmul_pair(hipStream_t s, const RowmulProblem<TA, TM, TO>& p0, const RowmulProblem<TA, TM, TO>& p1) {
  const RowmulProblem<TA, TM, TO>* pp[2] = {&p0, &p1};
  unsigned gx = 0, gy = 0, tiles = 0;
  for (const auto* p : pp) {
    if (p->rows < 0 || p->w < 0) return hipErrorInvalidValue;
    if (p->gpart != nullptr && p->w > 16) return hipErrorInvalidValue;  // the Gram epilogue needs whole rows in one tile
    const unsigned x = (unsigned)((p->rows + 15) / 16), y = (unsigned)((p->w + 15) / 16);
    gx = std::max(gx, x);
    gy = std::max(gy, y);
    tiles += x * y;
  }
  if (tiles == 0) return hipSuccess;
  if (tiles >= kTallMinTiles && p0.gpart == nullptr && p1.gpart == nullptr) {
    unsigned tx = 0, ty = 0;
    for (const auto* p : pp) {
      tx = std::max(tx, (unsigned)((p->rows + kTallRows - 1) / kTallRows));
      ty = std::max(ty, (unsigned)((p->w + kTallCols - 1) / kTallCols));
    }
    hipLaunchKernelGGL((k_rowmul_tall<TA, TM, TO>), dim3(tx, ty, 2), dim3(4 * kWave), 0, s, p0, p1);
    return hipGetLastError();
  }
  const dim3 grid(gx, gy, 2);
  if (tiles < 256)
    hipLaunchKernelGGL((k_rowmul<TA, TM, TO, 16>), grid, dim3(16 * kWave), 0, s, p0, p1);
  else
    hipLaunchKernelGGL((k_rowmul<TA, TM, TO, 4>), grid, dim3(4 * kWave), 0, s, p0, p1);
  return hipGetLastError();
}

template <class TA, class TM, class TO>
hipError_t launch_rowmul(hipStream_t s, int rows, int K, const TA* A, int lda, const TM* M, int ldm, TO* out, int ldo,
                         int w, double alpha, double beta, double* gpart) {
  if (rows == 0 || w == 0) return hipSuccess;
  if (gpart != nullptr && w > 16) return hipErrorInvalidValue;  // the Gram epilogue needs whole rows in one tile
  const RowmulProblem<TA, TM, TO> p{rows, K, A, lda, M, ldm, out, ldo, w, alpha, beta, gpart};
  RowmulProblem<TA, TM, TO> none = p;
  none.rows = 0;
  const dim3 grid((rows + 15) / 16, (w + 15) / 16, 1);
  if (grid.x * grid.y >= kTallMinTiles && gpart == nullptr) {
    hipLaunchKernelGGL((k_rowmul_tall<TA, TM, TO>), dim3((rows + kTallRows - 1) / kTallRows,
                       (w + kTallCols - 1) / kTallCols, 1), dim3(4 * kWave), 0, s, p, none);
    return hipGetLastError();
  }
  if (grid.x * grid.y < 256)
    hipLaunchKernelGGL((k_rowmul<TA, TM, TO, 16>), grid, dim3(16 * kWave), 0, s, p, none);
  else
    hipLaunchKernelGGL((k_rowmul<TA, TM, TO, 4>), grid, dim3(4 * kWave), 0, s, p, none);
  return hipGetLastError();
}

// A^T B over at most this many rows runs as one split of sixteen waves per 16 x 16 tile
constexpr int kTnDirectRows = 2048;

template <class TA, class TB>
hipError_t launch_tn_narrow(hipStream_t s, int rows, const TA* A, int lda, int na, const TB* B, int ldb, int nb,
                            double* out, int ldo, double* partial, int64_t partial_cap) {
  if (na == 0 || nb == 0) return hipSuccess;
  const int gx = (na + 15) / 16, gy = (nb + 15) / 16;
  if (rows <= kTnDirectRows) {
    hipLaunchKernelGGL((k_tn_narrow<TA, TB, 16>), dim3(gx, gy, 1), dim3(16 * kWave), 0, s, rows, A, lda, na, B, ldb, nb,
                       out, (int64_t)0, ldo, std::max(rows, 1));
    return hipGetLastError();
  }
  // enough workgroups to fill the chip: about 512 in total, at least 64 rows per split
  int splits = std::max(1, std::min(std::max(1, rows / 64), 512 / std::max(1, gx * gy)));
  while (splits > 1 && (int64_t)splits * na * nb > partial_cap) --splits;
  const int rps = (rows + splits - 1) / splits;
  hipLaunchKernelGGL((k_tn_narrow<TA, TB, 4>), dim3(gx, gy, splits), dim3(256), 0, s, rows, A, lda, na, B, ldb, nb,
                     partial, (int64_t)na * nb, nb, std::max(rps, 1));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tn_finish, dim3(grid1((int64_t)na * nb)), dim3(256), 0, s, partial, splits, na, nb, out, ldo);
  return hipGetLastError();
}

hipError_t launch_tn_finish(hipStream_t s, const double* partial, int splits, int na, int nb, double* out, int ldo) {
  if (na <= 0 || nb <= 0) return hipSuccess;
  if (splits <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tn_finish, dim3(grid1((int64_t)na * nb)), dim3(256), 0, s, partial, splits, na, nb, out, ldo);
  return hipGetLastError();
}

template <class T>
hipError_t launch_gram(hipStream_t s, int rows, const T* A, int lda, int na, double* G, int ldg, double* partial,
                       int64_t partial_cap) {
  (void)partial;
  (void)partial_cap;
  if (na == 0) return hipSuccess;
  // wide blocks over many rows: 64 x 64 LDS-staged tiles (16 x 16 tiles re-read every column
  // block na / 16 times, and their operand traffic dominates there)
  if ((int64_t)rows * na >= kGramTiledMin) return launch_gram_tn<T>(s, rows, A, lda, na, G, ldg);
  // from a few hundred columns on, 32 x 32 tiles (half the operand loads per product); below, the
  // 16 x 16 tiles spread more workgroups over the compute units
  if (na >= kGram32MinCols) {
    const int nt = (na + kGT2 - 1) / kGT2;
    hipLaunchKernelGGL(k_gram_tiles32<T>, dim3(nt * (nt + 1) / 2), dim3(kGram2Waves * kWave), 0, s, rows, A, lda, na,
                       G, ldg, nt);
    return hipGetLastError();
  }
  const int nt = (na + kGT - 1) / kGT;
  const int ntri = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(k_gram_tiles<T>, dim3(ntri), dim3(kGramWaves * kWave), 0, s, rows, A, lda, na, G, ldg, nt);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sumsq_cols(hipStream_t s, int rows, const T* A, int lda, int c0, int w, double* partial,
                             double* scal, int slot, const PostReq* post) {
  const int64_t total = (int64_t)rows * w;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (total + 255) / 256));
  hipLaunchKernelGGL(k_sumsq_cols<T>, dim3(nb), dim3(256), 0, s, rows, A, lda, c0, w, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finish(s, partial, nb, 1, 1, scal, slot, post);
}

template <class T>
hipError_t launch_sumsq(hipStream_t s, int64_t len, const T* v, double* partial, double* scal, int slot) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (len + 255) / 256));
  hipLaunchKernelGGL(k_sumsq<T>, dim3(nb), dim3(256), 0, s, len, v, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, partial, nb, 1, 1, scal, slot, nullptr, 0, nullptr, nullptr, 0u);
  return hipGetLastError();
}

template <class T>
hipError_t launch_colnorms(hipStream_t s, int rows, const T* A, int lda, int w, double* gram_scratch, double* partial,
                           int64_t partial_cap, double* out) {
  hipError_t e = launch_tn_narrow<T, T>(s, rows, A, lda, w, A, lda, w, gram_scratch, w, partial, partial_cap);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_sqrt, dim3(1), dim3(128), 0, s, gram_scratch, w, w, out);
  return hipGetLastError();
}

template <class TA, class TB>
hipError_t launch_tn_partial(hipStream_t s, int rows, const TA* A, int lda, int na, const TB* B, int ldb, int nb,
                             double* partial, int64_t partial_cap, int* splits_out) {
  *splits_out = 0;
  if (na == 0 || nb == 0) return hipSuccess;
  const int gx = (na + 15) / 16, gy = (nb + 15) / 16;
  if (rows <= kTnDirectRows && (int64_t)na * nb <= partial_cap) {  // one split
    hipLaunchKernelGGL((k_tn_narrow<TA, TB, 16>), dim3(gx, gy, 1), dim3(16 * kWave), 0, s, rows, A, lda, na, B, ldb, nb,
                       partial, (int64_t)na * nb, nb, std::max(rows, 1));
    *splits_out = 1;
    return hipGetLastError();
  }
  int splits = std::max(1, std::min(std::max(1, rows / 64), 512 / std::max(1, gx * gy)));
  while (splits > 1 && (int64_t)splits * na * nb > partial_cap) --splits;
  const int rps = (rows + splits - 1) / splits;
  hipLaunchKernelGGL((k_tn_narrow<TA, TB, 4>), dim3(gx, gy, splits), dim3(256), 0, s, rows, A, lda, na, B, ldb, nb,
                     partial, (int64_t)na * nb, nb, std::max(rps, 1));
  *splits_out = splits;
  return hipGetLastError();
}

hipError_t launch_block_chol(hipStream_t s, const double* gram, int ldg, int w, const double* prenorm,
                             double drop_tol, double dep_tol, double* Rout, int ldm, double* scal, int slot,
                             int wk_slot_in, int splits, int64_t sstride) {
  if (splits <= 0) return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_block_chol, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(kEigMax * (kEigMax + 1) * sizeof(double)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const size_t lds = (size_t)w * (w + 1) * sizeof(double);
  hipLaunchKernelGGL(k_block_chol, dim3(1), dim3(kBlockCholThreads), lds, s, gram, ldg, splits, sstride, w, prenorm,
                     drop_tol,
                     dep_tol, Rout, ldm, scal, slot, wk_slot_in);
  return hipGetLastError();
}

template <int WM, class T>
hipError_t set_trsm_attr() {
  static bool attr_set = false;
  if (attr_set) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_trsm_rows<WM, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(kEigMax * (kEigMax + 1) * sizeof(double)));
  if (e == hipSuccess) attr_set = true;
  return e;
}

template <class T>
hipError_t launch_trsm_rows(hipStream_t s, int rows, const T* X, int ldx, int w, const double* R, int ldr, T* out,
                            int ldo) {
  if (rows < 0 || w < 0 || w > kEigMax) return hipErrorInvalidValue;
  if (rows == 0 || w == 0) return hipSuccess;
  const size_t lds = (size_t)w * (w + 1) * sizeof(double);
  // one row per thread in 64-thread workgroups: a few hundred rows still occupy many CUs
  constexpr int kTB = 64;
  const unsigned g = (unsigned)((rows + kTB - 1) / kTB);
  hipError_t e;
  if (w <= 16) {
    if ((e = set_trsm_attr<16, T>()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_trsm_rows<16, T>), dim3(g), dim3(kTB), lds, s, rows, X, ldx, w, R, ldr, out, ldo);
  } else if (w <= 32) {
    if ((e = set_trsm_attr<32, T>()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_trsm_rows<32, T>), dim3(g), dim3(kTB), lds, s, rows, X, ldx, w, R, ldr, out, ldo);
  } else if (w <= 64) {
    if ((e = set_trsm_attr<64, T>()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_trsm_rows<64, T>), dim3(g), dim3(kTB), lds, s, rows, X, ldx, w, R, ldr, out, ldo);
  } else {
    if ((e = set_trsm_attr<kEigMax, T>()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_trsm_rows<kEigMax, T>), dim3(g), dim3(kTB), lds, s, rows, X, ldx, w, R, ldr, out, ldo);
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_chol_trsm(hipStream_t s, int rows, const T* X, int ldx, int w, const double* gram, int splits,
                            int64_t sstride, const double* prenorm, double drop_tol, double dep_tol, int wk_slot_in,
                            T* out, int ldo, double* gout, double* scal, int slot) {
  if (rows <= 0 || w <= 0 || w > kCholTrsmMaxCols || splits <= 0) return hipErrorInvalidValue;
  if (gout != nullptr && w > 32) return hipErrorInvalidValue;  // the Gram epilogue is for at most 32 columns
  const dim3 g((unsigned)((rows + kCholTrsmRows - 1) / kCholTrsmRows));
  if (w <= 16)
    hipLaunchKernelGGL((k_chol_trsm<16, T>), g, dim3(kCholTrsmThreads), 0, s, rows, X, ldx, w, gram, splits, sstride,
                       prenorm, drop_tol, dep_tol, wk_slot_in, out, ldo, gout, scal, slot);
  else if (w <= 32)
    hipLaunchKernelGGL((k_chol_trsm<32, T>), g, dim3(kCholTrsmThreads), 0, s, rows, X, ldx, w, gram, splits, sstride,
                       prenorm, drop_tol, dep_tol, wk_slot_in, out, ldo, gout, scal, slot);
  else if (w <= 64)
    hipLaunchKernelGGL((k_chol_trsm<64, T>), g, dim3(kCholTrsmThreads), 0, s, rows, X, ldx, w, gram, splits, sstride,
                       prenorm, drop_tol, dep_tol, wk_slot_in, out, ldo, gout, scal, slot);
  else
    hipLaunchKernelGGL((k_chol_trsm<96, T>), g, dim3(kCholTrsmThreads), 0, s, rows, X, ldx, w, gram, splits, sstride,
                       prenorm, drop_tol, dep_tol, wk_slot_in, out, ldo, gout, scal, slot);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sddmm_update(hipStream_t s, int nchunks, const int32_t* cstart, const int32_t* ccol,
                               const int32_t* rowidx, const T* a, const T* y, T* y_next, const T* Ut, const T* Vt,
                               int ld, int k, double delta, double* partial, int* nblocks, T* yT, int64_t ldy) {
  const int nb = std::max(1, (nchunks + 3) / 4);
  *nblocks = nb;
  constexpr int E = (int)(16 / sizeof(T));
  const int kv = (std::max(k, 1) + E - 1) / E;
  const size_t lds = (size_t)4 * kv * E * sizeof(T);
  if (lds > 160 * 1024 - 1024) return hipErrorInvalidValue;
  // the batch: the factor row's vectors up to eight, no loads beyond them for short rows
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               160 * 1024 - 1024);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(nb), dim3(256), lds, s, nchunks, cstart, ccol, rowidx, a, y, y_next, Ut, Vt, ld, k,
                       (T)delta, partial, yT, ldy);
    return hipGetLastError();
  };
  if (kv <= 1) return go(k_sddmm_update<T, 1>);
  if (kv <= 2) return go(k_sddmm_update<T, 2>);
  if (kv <= 4) return go(k_sddmm_update<T, 4>);
  return go(k_sddmm_update<T, 8>);
}

hipError_t launch_absdiff_sum(hipStream_t s, int64_t len, const double* x, const double* ref, double* partial,
                              double* scal, int slot) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (len + 255) / 256));
  hipLaunchKernelGGL(k_absdiff, dim3(nb), dim3(256), 0, s, len, x, ref, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finish(s, partial, nb, 1, 1, scal, slot);
}

// dst[0..count) = src[0..count) in host memory mapped into the device, then *flag = seq once every
// value is visible to the host (each thread's system-scope fence, the barrier, then thread 0's)
__global__ __launch_bounds__(256) void k_post(const double* __restrict__ src, int count, double* dst,
                                              unsigned* flag, unsigned seq) {
  post_to_host(src, count, dst, flag, seq);
}

hipError_t launch_post(hipStream_t s, const double* src, int count, double* dst_mapped, unsigned* flag_mapped,
                       unsigned seq) {
  if (count < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_post, dim3(1), dim3(256), 0, s, src, count, dst_mapped, flag_mapped, seq);
  return hipGetLastError();
}

hipError_t launch_finish(hipStream_t s, const double* partial, int nblocks, int stride, int nq, double* scal,
                         int slot, const PostReq* post) {
  const PostReq none;
  const PostReq& p = post ? *post : none;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, partial, nblocks, stride, nq, scal, slot, p.src, p.count, p.dst,
                     p.flag, p.seq);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sample(hipStream_t s, int64_t nq, const int32_t* qi, const int32_t* qj, const T* Ut, const T* Vt,
                         int ld, int k, int64_t m, int64_t n, double* out) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample<T>, dim3(grid1(nq)), dim3(256), 0, s, nq, qi, qj, Ut, Vt, ld, k, m, n, out);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mae_fused(hipStream_t s, int64_t nq, const int32_t* qi, const int32_t* qj, const T* Ut, const T* Vt,
                           int ld, int k, int64_t m, int64_t n, const double* ref, double* work, double* out) {
  if (nq <= 0) return hipErrorInvalidValue;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kMaeFusedBlocks, (nq + 255) / 256));
  hipLaunchKernelGGL(k_sample_absdiff<T>, dim3(nb), dim3(256), 0, s, nq, qi, qj, Ut, Vt, ld, k, m, n, ref, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, work, nb, 1, 1, work, kMaeFusedBlocks, nullptr, 0, nullptr,
                     nullptr, 0u);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_div_store, dim3(1), dim3(64), 0, s, work + kMaeFusedBlocks, (double)nq, out);
  return hipGetLastError();
}

template <class TS, class TD>
hipError_t launch_scale_copy(hipStream_t s, int64_t len, const TS* src, double alpha, TD* dst) {
  if (len == 0) return hipSuccess;
  hipLaunchKernelGGL((k_scale_copy<TS, TD>), dim3(grid1(len)), dim3(256), 0, s, len, src, alpha, dst);
  return hipGetLastError();
}

hipError_t launch_gather_perm(hipStream_t s, int64_t len, const int32_t* perm, const double* src, double* dst) {
  if (len == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_perm, dim3(grid1(len)), dim3(256), 0, s, len, perm, src, dst);
  return hipGetLastError();
}

template <class TS, class TD>
hipError_t launch_copy_cols(hipStream_t s, int rows, const TS* src, int lds_, TD* dst, int ldd, int w) {
  const int64_t work = (int64_t)rows * w;
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL((k_copy_cols<TS, TD>), dim3(grid1(work)), dim3(256), 0, s, rows, src, lds_, dst, ldd, w);
  return hipGetLastError();
}

// explicit instantiations for the two storage types
#define SVT_INST(T)                                                                                                   \
  template hipError_t launch_omega<T>(hipStream_t, T*, int, int, int, int, uint64_t, uint64_t, uint64_t);             \
  template hipError_t launch_seg_spmm<T, T>(hipStream_t, int, const int32_t*, const int32_t*, const int32_t*,        \
                                            const T*, const T*, int, T*, int, int, int64_t, int, const SegChunks*);   \
  template hipError_t launch_spmm_t_tiled<T, T>(hipStream_t, int, int, const int32_t*, const int32_t*, const T*,      \
                                                const T*, int, int, T*, int, double*, int64_t);                       \
  template hipError_t launch_tn_narrow<T, T>(hipStream_t, int, const T*, int, int, const T*, int, int, double*, int,  \
                                             double*, int64_t);                                                       \
  template hipError_t launch_tn_partial<T, T>(hipStream_t, int, const T*, int, int, const T*, int, int, double*,      \
                                              int64_t, int*);                                                         \
  template hipError_t launch_gram<T>(hipStream_t, int, const T*, int, int, double*, int, double*, int64_t);           \
  template hipError_t launch_sumsq_cols<T>(hipStream_t, int, const T*, int, int, int, double*, double*, int,          \
                                           const PostReq*);                                                            \
  template hipError_t launch_sumsq<T>(hipStream_t, int64_t, const T*, double*, double*, int);                         \
  template hipError_t launch_colnorms<T>(hipStream_t, int, const T*, int, int, double*, double*, int64_t, double*);   \
  template hipError_t launch_trsm_rows<T>(hipStream_t, int, const T*, int, int, const double*, int, T*, int);         \
  template hipError_t launch_chol_trsm<T>(hipStream_t, int, const T*, int, int, const double*, int, int64_t,          \
                                          const double*, double, double, int, T*, int, double*, double*, int);        \
  template hipError_t launch_sddmm_update<T>(hipStream_t, int, const int32_t*, const int32_t*, const int32_t*,       \
                                             const T*, const T*, T*, const T*, const T*, int, int, double, double*,   \
                                             int*, T*, int64_t);                                                      \
  template hipError_t launch_sample<T>(hipStream_t, int64_t, const int32_t*, const int32_t*, const T*, const T*, int, \
                                       int, int64_t, int64_t, double*);                                               \
  template hipError_t launch_mae_fused<T>(hipStream_t, int64_t, const int32_t*, const int32_t*, const T*, const T*,    \
                                          int, int, int64_t, int64_t, const double*, double*, double*);               \
  template hipError_t launch_scale_copy<T, T>(hipStream_t, int64_t, const T*, double, T*);                            \
  template hipError_t launch_copy_cols<T, T>(hipStream_t, int, const T*, int, T*, int, int);

SVT_INST(double)
SVT_INST(float)
#undef SVT_INST

template hipError_t launch_rowmul_pair<double, double, double>(hipStream_t, const RowmulProblem<double, double, double>&,
                                                               const RowmulProblem<double, double, double>&);
template hipError_t launch_rowmul<double, double, double>(hipStream_t, int, int, const double*, int, const double*,
                                                          int, double*, int, int, double, double, double*);
template hipError_t launch_rowmul_pair<float, double, float>(hipStream_t, const RowmulProblem<float, double, float>&,
                                                               const RowmulProblem<float, double, float>&);
template hipError_t launch_rowmul<float, double, float>(hipStream_t, int, int, const float*, int, const double*, int,
                                                        float*, int, int, double, double, double*);
template hipError_t launch_rowmul_pair<float, double, double>(hipStream_t, const RowmulProblem<float, double, double>&,
                                                               const RowmulProblem<float, double, double>&);
template hipError_t launch_rowmul<float, double, double>(hipStream_t, int, int, const float*, int, const double*, int,
                                                         double*, int, int, double, double, double*);
template hipError_t launch_tn_narrow<float, double>(hipStream_t, int, const float*, int, int, const double*, int, int,
                                                    double*, int, double*, int64_t);
template hipError_t launch_copy_cols<float, double>(hipStream_t, int, const float*, int, double*, int, int);
template hipError_t launch_copy_cols<double, float>(hipStream_t, int, const double*, int, float*, int, int);
template hipError_t launch_scale_copy<double, float>(hipStream_t, int64_t, const double*, double, float*);

// the BF16 form: a bfloat16 basis with float32 iterate, projections and factors
template hipError_t launch_seg_spmm<float, bf16>(hipStream_t, int, const int32_t*, const int32_t*, const int32_t*,
                                                 const float*, const bf16*, int, float*, int, int, int64_t, int,
                                                 const SegChunks*);
template hipError_t launch_spmm_t_tiled<float, bf16>(hipStream_t, int, int, const int32_t*, const int32_t*,
                                                     const float*, const bf16*, int, int, float*, int, double*,
                                                     int64_t);
template hipError_t launch_tn_narrow<bf16, float>(hipStream_t, int, const bf16*, int, int, const float*, int, int,
                                                  double*, int, double*, int64_t);
template hipError_t launch_tn_narrow<bf16, bf16>(hipStream_t, int, const bf16*, int, int, const bf16*, int, int,
                                                 double*, int, double*, int64_t);
template hipError_t launch_rowmul<bf16, double, float>(hipStream_t, int, int, const bf16*, int, const double*, int,
                                                       float*, int, int, double, double, double*);
template hipError_t launch_copy_cols<float, bf16>(hipStream_t, int, const float*, int, bf16*, int, int);

}  // namespace svt
