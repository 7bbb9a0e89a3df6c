// FP64 matrix multiply on the gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
//   C = alpha * op(A) * op(B) + beta * C      (column-major)
//
// Used for every dense contraction of the chain: the Cholesky trailing
// update, W = L^T J L, the skew rank-2k update of the tridiagonalisation,
// the block-reflector applications and the products with L.  Options:
//   c_uplo  0: full C;  1: lower triangle incl. diagonal;  2: strictly lower
//           (only tiles touching the requested triangle are launched)
//   a_tri   the stored A is lower triangular: the K loop skips its zeros
//   b_tri   the stored B is lower triangular
//
// Tiling: 64 x 64 C tile per 256-thread workgroup (4 wavefronts in a 2 x 2
// arrangement, 32 x 32 each = 2 x 2 MFMA blocks of 16 x 16), K step 16
// staged through LDS with a register prefetch of the next K slab.
#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;

struct GemmParams {
  int M, N, K;
  const double* A;
  long lda;
  const double* B;
  long ldb;
  double* C;
  long ldc;
  double alpha, beta;
  int c_uplo, a_tri, b_tri;
  int tiles_m, tiles_n;
};

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmParams p) {
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BN + PAD];

  int tm, tn;
  if (p.c_uplo) {
    tri_index(blockIdx.x, tm, tn);
  } else {
    tm = blockIdx.x % p.tiles_m;
    tn = blockIdx.x / p.tiles_m;
  }
  const int i0 = tm * BM, j0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;

  // K range that can hold non-zero products for this tile
  int kbeg = 0, kend = p.K;
  if (p.a_tri) {
    if (!TA) kend = min(kend, i0 + BM);
    else kbeg = max(kbeg, i0);
  }
  if (p.b_tri) {
    if (!TB) kbeg = max(kbeg, j0);
    else kend = min(kend, j0 + BN);
  }

  d4_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};

  // per-thread load coordinates (4 consecutive elements along the contiguous
  // direction of the stored operand)
  double ra[4], rb[4];
  auto load_a = [&](int k0) {
    if (!TA) {  // op(A)[i,k] = A[i + k*lda]; tile: 64 rows x 16 cols
      const int kk = tid >> 4, ii = (tid & 15) * 4;
      const int k = k0 + kk;
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + ii + q;
        ra[q] = (i < p.M && k < kend) ? p.A[(long)i + (long)k * p.lda] : 0.0;
      }
    } else {    // op(A)[i,k] = A[k + i*lda]; tile: 64 cols of A, 16 rows each
      const int ii = tid >> 2, kk = (tid & 3) * 4;
      const int i = i0 + ii;
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + kk + q;
        ra[q] = (i < p.M && k < kend) ? p.A[(long)k + (long)i * p.lda] : 0.0;
      }
    }
  };
  auto store_a = [&](int buf) {
    if (!TA) {
      const int kk = tid >> 4, ii = (tid & 15) * 4;
      for (int q = 0; q < 4; ++q) As[buf][kk][ii + q] = ra[q];
    } else {
      const int ii = tid >> 2, kk = (tid & 3) * 4;
      for (int q = 0; q < 4; ++q) As[buf][kk + q][ii] = ra[q];
    }
  };
  auto load_b = [&](int k0) {
    if (!TB) {  // op(B)[k,j] = B[k + j*ldb]; 64 cols of B, 16 rows each
      const int jj = tid >> 2, kk = (tid & 3) * 4;
      const int j = j0 + jj;
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + kk + q;
        rb[q] = (j < p.N && k < kend) ? p.B[(long)k + (long)j * p.ldb] : 0.0;
      }
    } else {    // op(B)[k,j] = B[j + k*ldb]; 16 cols of B, 64 rows each
      const int kk = tid >> 4, jj = (tid & 15) * 4;
      const int k = k0 + kk;
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + jj + q;
        rb[q] = (j < p.N && k < kend) ? p.B[(long)j + (long)k * p.ldb] : 0.0;
      }
    }
  };
  auto store_b = [&](int buf) {
    if (!TB) {
      const int jj = tid >> 2, kk = (tid & 3) * 4;
      for (int q = 0; q < 4; ++q) Bs[buf][kk + q][jj] = rb[q];
    } else {
      const int kk = tid >> 4, jj = (tid & 15) * 4;
      for (int q = 0; q < 4; ++q) Bs[buf][kk][jj + q] = rb[q];
    }
  };

  // align the start of the K loop to BK so that tiles stay aligned
  kbeg = (kbeg / BK) * BK;
  int buf = 0;
  if (kbeg < kend) {
    load_a(kbeg);
    load_b(kbeg);
    store_a(0);
    store_b(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      load_a(k0 + BK);
      load_b(k0 + BK);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[2], bf[2];
      for (int a = 0; a < 2; ++a) af[a] = As[buf][kr][wr * 32 + a * 16 + (lane & 15)];
      for (int b = 0; b < 2; ++b) bf[b] = Bs[buf][kr][wc * 32 + b * 16 + (lane & 15)];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (more) {
      store_a(buf ^ 1);
      store_b(buf ^ 1);
    }
    __syncthreads();
    buf ^= 1;
  }

  // epilogue: in a 16 x 16 f64 block, entry (i, j) lives in lane
  // 16 (i mod 4) + j, accumulator element i / 4
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int col = j0 + wc * 32 + b * 16 + (lane & 15);
      for (int v = 0; v < 4; ++v) {
        const int row = i0 + wr * 32 + a * 16 + (lane >> 4) + 4 * v;
        if (row >= p.M || col >= p.N) continue;
        if (p.c_uplo == 1 && row < col) continue;
        if (p.c_uplo == 2 && row <= col) continue;
        double* c = p.C + (long)row + (long)col * p.ldc;
        const double val = p.alpha * acc[a][b][v];
        *c = (p.beta == 0.0) ? val : val + p.beta * (*c);
      }
    }
}

}  // namespace

int gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
             long lda, const double* B, long ldb, double beta, double* C, long ldc, int c_uplo,
             int a_tri, int b_tri) {
  if (M <= 0 || N <= 0) return 0;
  GemmParams p;
  p.M = M;
  p.N = N;
  p.K = K < 0 ? 0 : K;
  p.A = A;
  p.lda = lda;
  p.B = B;
  p.ldb = ldb;
  p.C = C;
  p.ldc = ldc;
  p.alpha = alpha;
  p.beta = beta;
  p.c_uplo = c_uplo;
  p.a_tri = a_tri;
  p.b_tri = b_tri;
  p.tiles_m = (M + BM - 1) / BM;
  p.tiles_n = (N + BN - 1) / BN;
  long nblocks;
  if (c_uplo) {
    if (M != N) return set_hip_error(hipErrorInvalidValue, "gemm: triangular C must be square", __FILE__, __LINE__);
    nblocks = (long)p.tiles_m * (p.tiles_m + 1) / 2;
  } else {
    nblocks = (long)p.tiles_m * p.tiles_n;
  }
  dim3 grid((unsigned)nblocks), block(256);
  if (!ta && !tb) gemm_f64_kernel<false, false><<<grid, block, 0, s>>>(p);
  else if (!ta && tb) gemm_f64_kernel<false, true><<<grid, block, 0, s>>>(p);
  else if (ta && !tb) gemm_f64_kernel<true, false><<<grid, block, 0, s>>>(p);
  else gemm_f64_kernel<true, true><<<grid, block, 0, s>>>(p);
  BSE_LAUNCHED();
  return 0;
}

}  // namespace bse
