// Dense products on the matrix cores for the dense path of W = Y^T Q: when at least a quarter
// of the entries are observed, Y is kept as a dense transposed copy (zeros off Lambda) and
// Y^T Q becomes a plain dense product.  W is the transpose of the projection B of the sampled
// basis (Alg. 1, Sec. 2.1), formed on the SVT iterate in Alg. 2-4.
#include <type_traits>

#include "svt_internal.h"

namespace svt {

namespace {

// ------------------------------------------------------------------------------------------
// C = A B (row-major; A M x K, B K x N) in the storage precision: v_mfma_f32_16x16x4f32 for
// float (float accumulation), v_mfma_f64_16x16x4f64 for double.  Both take the A operand as
// A[l % 16][l / 16] and the B operand as B[l / 16][l % 16] in lane l; the f32 result holds rows
// 4 (l / 16) + v, the f64 result rows (l / 16) + 4 v, v = 0..3, of column l % 16.
//
// A workgroup owns one 64 x GN tile of C (GN = 32 or 48) and is KG groups of four waves; group g
// takes the 32-wide K chunks g, g + KG, g + 2 KG, ... (each wave 16 rows x GN columns, GN / 16
// matrix instructions per k-step sharing the A operand), staging its chunk in its own LDS area
// while its next DEPTH chunks are in flight in registers.  The groups' accumulators are added
// in group order at the end (deterministic).  Splitting K inside the workgroup keeps KG times
// more loads in flight per tile than one group alone: at the sizes of the basis (a few hundred
// columns) there are few tiles per compute unit, and one group per tile would leave every CU
// waiting on memory latency.  The launcher takes the tile width that puts the fewest tile
// columns on the busiest CU (one round of 256 tiles of 48 rather than two of 32, say).
//
// With few tiles (a basis of a hundred columns gives 64 over 1024 rows) the K range is also cut
// into ks contiguous parts, each a workgroup of its own on the same XCD as the tile's others; the
// parts write their partial tiles to a workspace and k_split_sum adds them in part order
// (deterministic), so four times the compute units share the loads.
//
// The tile grid is split into ga x gb rectangles (ga gb = 8, chosen by the launcher to balance the
// tiles and then to minimise the operand bytes each XCD reads), one per XCD: the hardware deals
// consecutive workgroups round-robin over the eight XCDs, so workgroup id goes to XCD id % 8 and
// takes tile id / 8 of that XCD's rectangle.  Each XCD's L2 then fetches only its rectangle's
// row blocks of A and column blocks of B, instead of every column block of B.
// ------------------------------------------------------------------------------------------
constexpr int kGM = 64, kGK = 32;
constexpr int kXcd = 8;

template <class T>
struct Mfma16;
template <>
struct Mfma16<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  __device__ static acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct Mfma16<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  __device__ static acc_t mma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// K groups per workgroup: 4 for float (1024 threads), 2 for double (512 threads); register
// prefetch depth: two chunks for float, one for double (two would spill)
template <class T>
constexpr int gemm_kgroups() {
  return sizeof(T) == 4 ? 4 : 2;
}
template <class T>
constexpr int gemm_depth() {
  return sizeof(T) == 4 ? 2 : 1;
}

// part i of n items cut into g nearly equal contiguous parts: first item and count
__host__ __device__ inline void split_range(int n, int g, int i, int* first, int* count) {
  const int base = n / g, rem = n % g;
  *first = i * base + (i < rem ? i : rem);
  *count = base + (i < rem ? 1 : 0);
}

template <class T, int GN, class TB>
__global__ __launch_bounds__(256 * gemm_kgroups<T>()) void k_gemm_nn(int M, int N, int K, const T* __restrict__ A,
                                                                     int lda, const TB* __restrict__ B, int ldb,
                                                                     T* __restrict__ C, int ldc, int tiles_m,
                                                                     int tiles_n, int ga, int tri, int ks) {
  using MM = Mfma16<T>;
  constexpr int KG = gemm_kgroups<T>(), DEPTH = gemm_depth<T>();
  constexpr int NT = GN / 16, BL = kGK * GN / 256;  // column blocks; B elements per thread and chunk
  constexpr int kAS = kGM * (kGK + 1), kBS = kGK * (GN + 1);
  static_assert((KG - 1) * 4 * NT * 256 <= KG * (kAS + kBS), "the reduction area must fit in the staging area");
  __shared__ T smem[KG * (kAS + kBS)];
  const int tid = threadIdx.x & 255, kg = threadIdx.x >> 8, lane = tid & (kWave - 1), wv = tid / kWave;
  // this XCD's rectangle of the tile grid, and this workgroup's tile in it (workgroups past the
  // rectangle's tiles exit; uniform over the workgroup)
  const int xcd = blockIdx.x % kXcd, slot = (blockIdx.x / kXcd) / ks, part = (blockIdx.x / kXcd) % ks;
  const int gb = kXcd / ga;
  int ra0, rac, cb0, cbc;
  split_range(tiles_m, ga, xcd / gb, &ra0, &rac);
  split_range(tiles_n, gb, xcd % gb, &cb0, &cbc);
  if (slot >= rac * cbc) return;
  if (ks > 1) {  // part `part` of the K range writes its partial tile to its own M x N slice of C (ld N)
    C += (int64_t)part * M * N;
    ldc = N;
  }
  const int m0 = (ra0 + slot / cbc) * kGM, n0 = (cb0 + slot % cbc) * GN;
  T* As = smem + kg * (kAS + kBS);  // [kGM][kGK + 1]
  T* Bs = As + kAS;                  // [kGK][GN + 1]
  // global -> register staging, DEPTH chunks: A chunk 64 x 32 (8 per thread), B chunk 32 x GN
  T ra[DEPTH][8], rb[DEPTH][BL];
  auto load_chunk = [&](auto P, int k0) {
    constexpr int p = decltype(P)::value;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + u * 256, i = e / kGK, kk = e % kGK;
      const int gi = m0 + i, gk = k0 + kk;
      ra[p][u] = (gi < M && gk < K) ? A[(int64_t)gi * lda + gk] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < BL; ++u) {
      const int e = tid + u * 256, kk = e / GN, j = e % GN;
      const int gk = k0 + kk, gj = n0 + j;
      rb[p][u] = (gk < K && gj < N) ? (T)B[(int64_t)gk * ldb + gj] : (T)0;
    }
  };
  auto store_chunk = [&](auto P) {
    constexpr int p = decltype(P)::value;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + u * 256;
      As[(e / kGK) * (kGK + 1) + e % kGK] = ra[p][u];
    }
#pragma unroll
    for (int u = 0; u < BL; ++u) {
      const int e = tid + u * 256;
      Bs[(e / GN) * (GN + 1) + e % GN] = rb[p][u];
    }
  };
  typename MM::acc_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = typename MM::acc_t{0, 0, 0, 0};
  const int ar = wv * 16 + (lane & 15), kl = lane >> 4, bc = lane & 15;
  // a lower-triangular A (tri 1) or upper-triangular B (tri 2) holds zeros past the tile's diagonal: the
  // K chunks beyond it are skipped (the sums over the others are unchanged)
  const int Keff = tri == 1 ? min(K, m0 + kGM) : (tri == 2 ? min(K, n0 + GN) : K);
  int c_first = 0, nchunk = (Keff + kGK - 1) / kGK;
  if (ks > 1) {  // this part's chunks [c_first, nchunk)
    int cnt;
    split_range(nchunk, ks, part, &c_first, &cnt);
    nchunk = c_first + cnt;
  }
  const int rounds = (nchunk - c_first + KG - 1) / KG;
  // one round: stage chunk c from register buffer P, refill P with chunk c + DEPTH KG, multiply
  auto round = [&](auto P, int c) {
    __syncthreads();  // the previous chunk has been consumed
    if (c < nchunk) store_chunk(P);
    __syncthreads();
    if (c + DEPTH * KG < nchunk) load_chunk(P, (c + DEPTH * KG) * kGK);
    if (c < nchunk) {
#pragma unroll
      for (int ks = 0; ks < kGK / 4; ++ks) {
        const T a = As[ar * (kGK + 1) + ks * 4 + kl];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = MM::mma(a, Bs[(ks * 4 + kl) * (GN + 1) + 16 * t + bc], acc[t]);
      }
    }
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, DEPTH - 1>;
  int c = c_first + kg;
  if (c < nchunk) load_chunk(B0{}, c * kGK);
  if constexpr (DEPTH == 2) {
    if (c + KG < nchunk) load_chunk(B1{}, (c + KG) * kGK);
  }
  for (int rd = 0; rd < rounds; rd += DEPTH) {  // rounds is uniform over the workgroup
    round(B0{}, c);
    c += KG;
    if constexpr (DEPTH == 2) {
      if (rd + 1 < rounds) {
        round(B1{}, c);
        c += KG;
      }
    }
  }
  // add the groups' accumulators in group order; the staging area is reused
  __syncthreads();
  if (kg > 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) smem[((kg - 1) * 4 * NT + t * 4 + v) * 256 + tid] = acc[t][v];
  }
  __syncthreads();
  if (kg > 0) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = m0 + wv * 16 + MM::row(lane, v);
    if (row >= M) continue;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = n0 + 16 * t + bc;
      T sum = acc[t][v];
#pragma unroll
      for (int g = 1; g < KG; ++g) sum += smem[((g - 1) * 4 * NT + t * 4 + v) * 256 + tid];
      if (col < N) C[(int64_t)row * ldc + col] = sum;
    }
  }
}

// C[i][j] = sum over the ks partial products (M x N slices of P, in part order)
// With npart, also this workgroup's sum of squares of C (a fixed shuffle tree, then the four waves in
// order) in npart[blockIdx.x].
template <class T>
__global__ __launch_bounds__(256) void k_split_sum(int M, int N, int ks, const T* __restrict__ P, T* __restrict__ C,
                                                   int ldc, double* __restrict__ npart) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x, mn = (int64_t)M * N;
  double sq = 0.0;
  if (e < mn) {
    T sum = P[e];
    for (int q = 1; q < ks; ++q) sum += P[q * mn + e];
    C[(e / N) * ldc + e % N] = sum;
    sq = (double)sum * (double)sum;
  }
  if (npart == nullptr) return;  // uniform
  __shared__ double red[4];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) sq += __shfl_xor(sq, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = sq;
  __syncthreads();
  if (threadIdx.x == 0) npart[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);  // 256 threads
}

// yT[j * ldy + i] = y at CSC position p = (i, j): the dense transposed copy of Y on Lambda (the
// entries outside Lambda stay zero from set-up); one wave per column
template <class T>
__global__ __launch_bounds__(256) void k_scatter_dense_t(int n, const int32_t* __restrict__ colptr,
                                                         const int32_t* __restrict__ rowidx, const T* __restrict__ y,
                                                         T* __restrict__ yT, int64_t ldy) {
  const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (j >= n) return;
  for (int p = colptr[j] + lane; p < colptr[j + 1]; p += kWave) yT[(int64_t)j * ldy + rowidx[p]] = y[p];
}

}  // namespace

template <class T, class TB>
hipError_t launch_gemm_nn(hipStream_t s, int M, int N, int K, const T* A, int lda, const TB* B, int ldb, T* C, int ldc,
                          int tri, T* work, int64_t work_elems, const NormReq* nrm, int* nparts) {
  if (nparts) *nparts = 0;
  if (M == 0 || N == 0) return hipSuccess;
  if (M < 0 || N < 0 || K < 0) return hipErrorInvalidValue;
  const int tm = (M + kGM - 1) / kGM;
  // tile columns on the busiest of the 256 CUs, rounds of 256 tiles: 48-wide tiles when that is
  // fewer than with 32-wide ones
  auto load = [&](int gn) { return (int64_t)((tm * ((N + gn - 1) / gn) + 255) / 256) * gn; };
  const int gn = load(48) < load(32) ? 48 : 32;
  const int tn = (N + gn - 1) / gn;
  // the XCD rectangles: fewest tiles on the busiest XCD, then fewest operand bytes per XCD.  With a
  // triangular operand the work of a tile grows with its row block (tri 1) or column block (tri 2):
  // every XCD then takes all of those blocks, so the heavy tiles are spread over the eight
  int ga = 1;
  int64_t best_tiles = -1, best_bytes = 0;
  for (int g = 1; g <= kXcd; g *= 2) {
    if ((tri == 1 && g != 1) || (tri == 2 && g != kXcd)) continue;
    const int rows = (tm + g - 1) / g, cols = (tn + kXcd / g - 1) / (kXcd / g);
    const int64_t tiles = (int64_t)rows * cols;
    const int64_t bytes = (int64_t)rows * kGM * sizeof(T) + (int64_t)cols * gn * sizeof(TB);
    if (best_tiles < 0 || tiles < best_tiles || (tiles == best_tiles && bytes < best_bytes)) {
      best_tiles = tiles;
      best_bytes = bytes;
      ga = g;
    }
  }
  // K parts: as many (up to four) as keep the grid within one round of 256 workgroups while every
  // K group of a part still gets two chunks, when the workspace holds the partial products
  int ks = 1;
  const int64_t nchunk = (K + kGK - 1) / kGK, mn = (int64_t)M * N;
  while (tri == 0 && ks < 4 && (int64_t)tm * tn * ks * 2 <= 256 && nchunk >= (int64_t)ks * 2 * 2 * gemm_kgroups<T>() &&
         work != nullptr && mn * ks * 2 <= work_elems)
    ks *= 2;
  T* out = ks > 1 ? work : C;
  const dim3 grid((unsigned)(best_tiles * kXcd * ks));
  if (gn == 48)
    hipLaunchKernelGGL((k_gemm_nn<T, 48, TB>), grid, dim3(256 * gemm_kgroups<T>()), 0, s, M, N, K, A, lda, B, ldb,
                       out, ldc, tm, tn, ga, tri, ks);
  else
    hipLaunchKernelGGL((k_gemm_nn<T, 32, TB>), grid, dim3(256 * gemm_kgroups<T>()), 0, s, M, N, K, A, lda, B, ldb,
                       out, ldc, tm, tn, ga, tri, ks);
  if (ks > 1) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = (mn + 255) / 256;
    const bool fuse = nrm != nullptr && nparts != nullptr && nb <= nrm->cap;
    hipLaunchKernelGGL(k_split_sum<T>, dim3((unsigned)nb), dim3(256), 0, s, M, N, ks, work, C, ldc,
                       fuse ? nrm->partial : nullptr);
    if (fuse) *nparts = (int)nb;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_scatter_dense_t(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx, const T* y, T* yT,
                                  int64_t ldy) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_dense_t<T>, dim3((n + 3) / 4), dim3(256), 0, s, n, colptr, rowidx, y, yT, ldy);
  return hipGetLastError();
}

#define SVT_GEMM_INST(T)                                                                                       \
  template hipError_t launch_gemm_nn<T, T>(hipStream_t, int, int, int, const T*, int, const T*, int, T*, int,   \
                                           int, T*, int64_t, const NormReq*, int*);                             \
  template hipError_t launch_scatter_dense_t<T>(hipStream_t, int, const int32_t*, const int32_t*, const T*, T*, \
                                                int64_t);

SVT_GEMM_INST(double)
SVT_GEMM_INST(float)
template hipError_t launch_gemm_nn<float, bf16>(hipStream_t, int, int, int, const float*, int, const bf16*, int, float*,
                                                int, int, float*, int64_t, const NormReq*, int*);

}  // namespace svt
