// Gram matrix G = A^T A of a wide block over many rows on the f64 matrix cores.
#include "svt_internal.h"

namespace svt {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
__device__ inline dbl4 mfma_f64(double a, double b, dbl4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Tile of workgroup id when `total` tiles are dealt round-robin over the eight XCDs (the
// hardware's order for consecutive workgroups): XCD x receives the contiguous range of tiles
// starting at x * (total / 8) + min(x, total % 8).
__device__ inline int xcd_range_tile(int id, int total) {
  const int x = id % 8, slot = id / 8, per = total / 8, rem = total % 8;
  return x * per + min(x, rem) + slot;
}

// ------------------------------------------------------------------------------------------
// Gram matrix G = A^T A (A rows x na, row-major, float or double; G in double) for wide blocks
// over many rows: the Gram step of the projected SVD (Alg. 1 on B B^T, with W = B^T; Alg. 3
// reuses it).  A workgroup of four waves owns one 64 x 64 tile of the upper triangle (tiles
// ti <= tj); each wave accumulates a 32 x 32 quarter as 2 x 2 v_mfma_f64_16x16x4f64 blocks.  The
// rows are taken in 32-row chunks: a chunk of both column blocks is converted to double and
// staged in LDS (row stride kQS = 80 doubles: the four k rows one matrix instruction reads fall
// on disjoint bank halves) while the next chunk is loaded into registers.  A diagonal tile
// stages one block; off-diagonal tiles also write the mirrored tile.
// ------------------------------------------------------------------------------------------
constexpr int kQT = 64, kQK = 32, kQS = 80;
constexpr int kQLoads = kQK * kQT / 256;  // elements of one block per thread and chunk

template <class T>
__global__ __launch_bounds__(256) void k_gram_tn(int rows, const T* __restrict__ A, int lda, int na,
                                                 double* __restrict__ G, int ldg, int nt) {
  __shared__ double As[kQK * kQS], Bs[kQK * kQS];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  // upper-triangular tile pair (ti <= tj) of this workgroup; tiles of one row block are dealt
  // to one XCD in a contiguous range
  int t = xcd_range_tile(blockIdx.x, gridDim.x), ti = 0;
  while (t >= nt - ti) {
    t -= nt - ti;
    ++ti;
  }
  const int tj = ti + t;
  const bool diag = ti == tj;
  const int a0 = ti * kQT, b0 = tj * kQT;
  const double* Bsrc = diag ? As : Bs;
  T ra[kQLoads], rb[kQLoads];
  auto load_chunk = [&](int r0) {
#pragma unroll
    for (int u = 0; u < kQLoads; ++u) {
      const int e = tid + u * 256, k = e / kQT, i = e % kQT;
      const int row = r0 + k;
      ra[u] = (row < rows && a0 + i < na) ? A[(int64_t)row * lda + a0 + i] : (T)0;
      rb[u] = (!diag && row < rows && b0 + i < na) ? A[(int64_t)row * lda + b0 + i] : (T)0;
    }
  };
  dbl4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int wy = wv >> 1, wx = wv & 1, kl = lane >> 4, cl = lane & 15;
  const int nchunk = (rows + kQK - 1) / kQK;
  if (nchunk > 0) load_chunk(0);
  for (int c = 0; c < nchunk; ++c) {  // nchunk is uniform over the workgroup
    __syncthreads();                  // the previous chunk has been consumed
#pragma unroll
    for (int u = 0; u < kQLoads; ++u) {
      const int e = tid + u * 256, k = e / kQT, i = e % kQT;
      As[k * kQS + i] = (double)ra[u];
      if (!diag) Bs[k * kQS + i] = (double)rb[u];
    }
    __syncthreads();
    if (c + 1 < nchunk) load_chunk((c + 1) * kQK);
#pragma unroll
    for (int ks = 0; ks < kQK / 4; ++ks) {
      const int k = ks * 4 + kl;
      double a[2], b[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        a[q] = As[k * kQS + wy * 32 + q * 16 + cl];
        b[q] = Bsrc[k * kQS + wx * 32 + q * 16 + cl];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma_f64(a[bi], b[bj], acc[bi][bj]);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ra_ = a0 + wy * 32 + bi * 16 + kl + 4 * v, cb = b0 + wx * 32 + bj * 16 + cl;
        if (ra_ < na && cb < na) {
          G[(int64_t)ra_ * ldg + cb] = acc[bi][bj][v];
          if (!diag) G[(int64_t)cb * ldg + ra_] = acc[bi][bj][v];
        }
      }
}

}  // namespace

int gram_tn_tiles(int na) {
  const int nt = (na + kQT - 1) / kQT;
  return nt * (nt + 1) / 2;
}

template <class T>
hipError_t launch_gram_tn(hipStream_t s, int rows, const T* A, int lda, int na, double* G, int ldg) {
  if (na == 0) return hipSuccess;
  if (rows < 0 || na < 0) return hipErrorInvalidValue;
  const int nt = (na + kQT - 1) / kQT;
  hipLaunchKernelGGL(k_gram_tn<T>, dim3(gram_tn_tiles(na)), dim3(256), 0, s, rows, A, lda, na, G, ldg, nt);
  return hipGetLastError();
}

template hipError_t launch_gram_tn<double>(hipStream_t, int, const double*, int, int, double*, int);
template hipError_t launch_gram_tn<float>(hipStream_t, int, const float*, int, int, double*, int);

}  // namespace svt
